"""Writes generator_digests.json: sha256 of the seeded synthetic inputs, so a
change to a generator (which would silently change every corpus, compressed
stream and measurement) fails the CPU suite.  Calls only the generators."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402


def digests() -> dict:
    d = {
        "zipf_text(1 MiB)": synth.sha256(synth.zipf_text(1 << 20)),
        "zipf_text(64 KiB at 3 MiB + 17)": synth.sha256(synth.zipf_text(1 << 16, off=(3 << 20) + 17)),
        "csv_rows(1 MiB)": synth.sha256(synth.csv_rows(1 << 20)),
        "csv_rows(64 KiB at 5 MiB + 3)": synth.sha256(synth.csv_rows(1 << 16, off=(5 << 20) + 3)),
    }
    seqs, lits = synth.nesting_tokens(640, 4)
    d["nesting_tokens(640, 4)"] = synth.sha256(np.frombuffer(seqs.tobytes() + lits, np.uint8))
    seqs, lits = synth.random_tokens(2000, 3)
    d["random_tokens(2000, 3)"] = synth.sha256(np.frombuffer(seqs.tobytes() + lits, np.uint8))
    d["batch_mix()"] = synth.sha256(np.frombuffer(json.dumps(synth.batch_mix()).encode(), np.uint8))
    d["request_mix(2000)"] = synth.sha256(np.frombuffer(json.dumps(synth.request_mix(2000)).encode(), np.uint8))
    return d


if __name__ == "__main__":
    with open(os.path.join(HERE, "generator_digests.json"), "w") as f:
        json.dump(digests(), f, indent=1, sort_keys=True)
        f.write("\n")

// Host-side pieces shared by the C ABI's source files (not part of the ABI).
#pragma once
#include <stdint.h>

#include "../../include/gompresso.h"

// The context's device word that records the first non-zero block status of
// its launches (read and cleared by gmp_poll), and its device.
int32_t* gmp_ctx_first_err_word(gmp_ctx* ctx);
int gmp_ctx_device(gmp_ctx* ctx);

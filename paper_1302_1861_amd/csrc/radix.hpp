// One stable pass of the LSD radix sort of psl_build, used on its own as a
// stable partition by an 8-bit digit.
#pragma once

#include "common.hpp"

namespace psl {

// Workspace of radix_pass over n items.
size_t radix_pass_ws_bytes(int64_t n);

// (keys_in, idx_in)[0 .. n) -> (keys_out, idx_out), grouped by the digit
// (key >> shift) & 255 in ascending order, input order kept within a digit.
// digit_start (device uint32 [256], optional) receives the first output
// index of each digit (so digit_start[d] counts the items below digit d).
psl_status radix_pass(const uint32_t *keys_in, const uint32_t *idx_in,
                      int64_t n, int shift, uint32_t *keys_out,
                      uint32_t *idx_out, uint32_t *digit_start, void *ws,
                      hipStream_t st);

}  // namespace psl

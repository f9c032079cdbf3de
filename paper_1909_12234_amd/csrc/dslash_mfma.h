// Matrix-core Wilson-Dirac operator for 16-bit storage (dslash_mfma.hip).
#pragma once
#include "lqt_internal.h"

namespace lqt {

// true when every byte offset of a group of 4R right-hand sides fits 32 bits
bool dslash_mf_fits(const Geom& g, int R, long long in_stride, long long out_stride);
// out = op(in) for nrhs fields (LQT_F16 or LQT_BF16), tiling t (t.rhs_per_thread = groups of
// 4 right-hand sides per lane, 1 or 2; t.block 64/128/256; t.chunk as the vector kernel)
void dslash_mf(lqt_ctx* c, int prec, int op, const void* in, void* out, int nrhs, long long in_stride,
               long long out_stride, const Tuned& t, double shift, double scale);

}  // namespace lqt

// FP64 MFMA tall-skinny products (device-layout FP64 fields, results on the device).
#pragma once
#include "lqt_internal.h"

namespace lqt {

// C[a][b] = x_a^+ y_b  (ka x kb, row-major)
// n = vector length (default: a fine field, 12 V)
void gemm_gram(lqt_ctx* c, const double2* X, int ka, const double2* Y, int kb, double2* C_dev, long long n = -1);
// C = X^+ Y for vectors of length n into caller buffers, with no allocation and no timer:
// nc chunks of the contraction (nc <= n / 4), partial tiles in part (nc * ka * kb entries,
// every entry read is written first), C_dev ka * kb entries; launches on stream st
void gemm_gram_into(hipStream_t st, const double2* X, int ka, const double2* Y, int kb, long long n, int nc,
                    double2* part, double2* C_dev);
// C_up[a][j] = x_a^+ P_+ z_j, C_dn[a][j] = x_a^+ P_- z_j for probes j0 .. j0+s-1
void gemm_probes(lqt_ctx* c, const double2* X, int ka, uint64_t seed, long long j0, int s, double2* Cup_dev,
                 double2* Cdn_dev);
// y_b = beta y_b + alpha sum_a x_a C[a][b]; Y must not overlap X
void gemm_combine(lqt_ctx* c, const double2* X, int ka, const double2* C_dev, int kb, double beta, double alpha,
                  double2* Y, long long n = -1);

}  // namespace lqt

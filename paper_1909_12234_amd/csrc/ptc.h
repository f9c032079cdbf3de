// Gauge-equivariant parallel-transport network (right preconditioner).
#pragma once
#include <vector>

#include "lqt_internal.h"

namespace lqt {

constexpr int NL = 4;     // layers
extern const int FEATS[5];  // features per layer boundary: 4 -> 8 -> 8 -> 8 -> 4
int ptc_weight_count();     // complex weights of the 4 layers
// set the FP32 master weights (2 * ptc_weight_count() floats) and the device copy
void ptc_set(lqt_ctx* c, const float* w, bool round_bf16);
// out = M(in) for nrhs fields in storage S (device layout), FP32 arithmetic
template <typename S>
void ptc_apply(lqt_ctx* c, const S* in, S* out, int nrhs);
// sum over pairs of ||M r - e||^2 / ||e||^2 and its gradient with respect to conj(W)
double ptc_loss_grad(lqt_ctx* c, const double2* r, const double2* e, int np, const float* Wh,
                     std::vector<double>& grad, const std::vector<double>& enorm2);
// r = A e for np error fields e, then ptc_loss_grad over the pairs (r, e)
double ptc_pairs_loss_grad(lqt_ctx* c, const double2* e, double2* r, int np, const float* Wh,
                           std::vector<double>& grad);

}  // namespace lqt

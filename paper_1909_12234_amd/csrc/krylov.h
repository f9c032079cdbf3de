// Device state of a batch of restarted GMRES cycles (one entry per slot).
#pragma once
#include "lqt_internal.h"

namespace lqt {

constexpr int KRY_MAXM = 64;  // largest restart length

struct KryState {
    int m;            // restart length
    double2* H;       // [slot][(m+1)*m]  Hessenberg, overwritten by its QR factor
    double* cs;       // [slot][m]        Givens cosines
    double2* sn;      // [slot][m]        Givens sines
    double2* g;       // [slot][m+1]      rotated right-hand side
    double* sc;       // [slot][m+1]      scale of each stored basis vector
    double2* alpha;   // [slot][m+1]      update coefficients of the current step
    double2* y;       // [slot][m+1]      least-squares solution
    double2* beta;    // [slot][m+1]      y_i * sc_i
    double* fac;      // [slot]           write scale of the current step
    double* nu;       // [slot]
    double* est;      // [slot]           Arnoldi residual estimate |g_{k}|
    double* target;   // [slot]           absolute residual target of the cycle
    int* kdim;        // [slot]           steps taken in the current cycle
    int* frozen;      // [slot]           1 once the cycle of the slot has ended
};

// storage S <-> FP64 over total complex entries of the same layout
template <typename S>
void fields_to_f64(lqt_ctx* c, const S* in, double2* out, long long total);
template <typename S>
void fields_from_f64(lqt_ctx* c, const double2* in, S* out, long long total);
template <typename S>
void kry_dots(lqt_ctx* c, const void* Vb, long long vstride, int j, int ns, double2* part);
template <typename S>
void kry_update(lqt_ctx* c, void* Vb, long long vstride, int j, int ns, const KryState& st, int scale, double* part);
template <typename S>
void kry_xupdate(lqt_ctx* c, double2* x, const int* act, const void* Zb, long long zstride, int ns,
                 const KryState& st);
template <typename S>
void kry_start(lqt_ctx* c, void* V0, const double2* r, const int* src, const double* rn2, int ns);
// nsb = partial-sum blocks per slot of the preceding dot / update pass (kry_blocks<S>)
template <typename S>
int kry_blocks(const lqt_ctx* c);
void kry_finish(lqt_ctx* c, const double2* part, int nsb, int j, int ns, const KryState& st, int pass);
void kry_norm_givens(lqt_ctx* c, const double* part, int nsb, int j, int ns, const KryState& st);
void kry_backsolve(lqt_ctx* c, int ns, const KryState& st);
// s-step cycle end with the residual carried in the basis: x[act[q]] += K_s beta and
// k_0 <- (r - A K_s beta) sqrt(N)/est; rn2[q] = |r - A K_s beta|^2 (part: ns *
// kry_carry_blocks<S> doubles of workspace)
template <typename S>
int kry_carry_blocks(const lqt_ctx* c);
template <typename S>
void kry_sstep_carry(lqt_ctx* c, double2* x, const int* act, void* Kb, long long kstride, int ns, const KryState& st,
                     double theta, double sigma, double* part, double* rn2);
// cycle state of slots starting from the carried residual
void kry_start_state_carry(lqt_ctx* c, const KryState& st, const double* target_abs, int ns);
void kry_start_state(lqt_ctx* c, const KryState& st, const int* src, const double* rn2, const double* target_abs,
                     int ns);
// s-step cycle end (vectors k_0..k_s of ns slots, A k_i = k_{i+1}/sigma + theta k_i): Gram,
// Cholesky, least squares; leaves the update coefficients in st.beta and kdim = steps used
template <typename S>
void sstep_finish(lqt_ctx* c, const void* Vb, long long vstride, int s, int ns, const KryState& st, double theta,
                  double sigma, DBuf& work);

}  // namespace lqt

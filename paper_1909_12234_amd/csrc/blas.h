// FP64 field BLAS and probe kernels (device layout [field][comp][site]).
#pragma once
#include "lqt_internal.h"

namespace lqt {

void norm2_fields(lqt_ctx* c, const double2* x, int nf, double* out_dev);
void dot_fields(lqt_ctx* c, const double2* x, const double2* y, int nf, double2* out_dev);
void probes_gen(lqt_ctx* c, uint64_t seed, long long j0, int nprobes, double2* out);
// partition probe vectors p0 .. p0+nvec-1 (hp probing signs, dilution into the 12
// spin-colour components when dilute) of a single-lattice context
void partition_probes_gen(lqt_ctx* c, uint64_t seed, long long p0, int nvec, int hp, int dilute, double2* out);
// LQT_EINVAL unless (hp_vectors, dilute) is a valid partition for the context's lattice
void check_partition(const lqt_ctx* c, int hp_vectors, int dilute);
// z_j^T y_j for nprobes fields; per_lattice: out_dev[j * nlat + k] over the sites of lattice k
void probe_dots(lqt_ctx* c, uint64_t seed, long long j0, const double2* y, int nprobes, double2* out_dev,
                bool per_lattice = false);
// out_dev[f * nlat + k] = |x_f|^2 over the sites of lattice k
void norm2_lattices(lqt_ctx* c, const double2* x, int nf, double* out_dev);
// out_dev[f * nlat + k] = sum of part[f * nparts + q] over the 256-site blocks q of lattice k
void sum_partials_lattices(lqt_ctx* c, const double* part, int nparts, int nf, double* out_dev);
void gamma5_fields(lqt_ctx* c, double2* x, int nf);
bool has_nonfinite(lqt_ctx* c, const double* p, size_t n);

}  // namespace lqt

namespace lqt {
void gaussian_fields(lqt_ctx* c, uint64_t seed, long long n, int nf, double2* out);
// out[f] = |W_f - theta_f Q_f|^2 for nf vectors of length n
void eig_residual_norms(lqt_ctx* c, const double2* W, const double2* Q, const double* theta_dev, long long n, int nf,
                        double* out_dev);
}  // namespace lqt

// Entry points whose implementation is not in this build yet: they fail with LQT_EINVAL
// and say so, so the exported C-ABI is complete and callers get a clear error.
#include "lqt_internal.h"

#define LQT_PENDING(c)                                              \
    do {                                                            \
        if (c) ((lqt_ctx*)(c))->err = std::string(__func__) + " is not implemented in this build"; \
        return LQT_EINVAL;                                          \
    } while (0)

extern "C" {

int lqt_basis_eig(lqt_ctx* c, int, double, double, const lqt_solver_opts*, lqt_basis**) { LQT_PENDING(c); }
int lqt_basis_prolongator(lqt_ctx* c, const int*, int, int, double, int, const lqt_solver_opts*, lqt_basis**) {
    LQT_PENDING(c);
}
int lqt_basis_from_vectors(lqt_ctx* c, const double*, int, lqt_basis**) { LQT_PENDING(c); }
int lqt_basis_eigenvalues(const lqt_basis*, double*, int*) { return LQT_EINVAL; }
int lqt_basis_vectors(const lqt_basis*, double*) { return LQT_EINVAL; }
void lqt_basis_free(lqt_basis*) {}
int lqt_precond_set(lqt_ctx* c, const void*, size_t) { LQT_PENDING(c); }
int lqt_precond_get(lqt_ctx* c, void*, size_t) { LQT_PENDING(c); }
int lqt_precond_apply(lqt_ctx* c, const double*, double*, int) { LQT_PENDING(c); }
int lqt_precond_train(lqt_ctx* c, int, uint64_t, const lqt_train_opts*, double*) { LQT_PENDING(c); }
int lqt_trace(lqt_ctx* c, const lqt_basis*, int, int, uint64_t, double, const lqt_solver_opts*, lqt_trace_result*,
              double*, double*) {
    LQT_PENDING(c);
}
int lqt_gram(lqt_ctx* c, const double*, int, const double*, int, double*) { LQT_PENDING(c); }
int lqt_project_probes(lqt_ctx* c, const double*, int, uint64_t, long long, int, double*, double*) {
    LQT_PENDING(c);
}
int lqt_combine(lqt_ctx* c, const double*, int, const double*, int, double, double, double*) { LQT_PENDING(c); }
int lqt_restrict(lqt_ctx* c, const lqt_basis*, const double*, double*, int) { LQT_PENDING(c); }
int lqt_prolong(lqt_ctx* c, const lqt_basis*, const double*, double*, int) { LQT_PENDING(c); }
int lqt_prolongator_get(const lqt_basis*, double*, long long*) { return LQT_EINVAL; }
int lqt_basis_prolongator_from(lqt_ctx* c, const int*, int, const double*, lqt_basis**) { LQT_PENDING(c); }

}  // extern "C"

// Entry points whose implementation is not in this build yet: they fail with LQT_EINVAL
// and say so, so the exported C-ABI is complete and callers get a clear error.
#include "lqt_internal.h"
#include "prolong.h"

#define LQT_PENDING(c)                                              \
    do {                                                            \
        if (c) ((lqt_ctx*)(c))->err = std::string(__func__) + " is not implemented in this build"; \
        return LQT_EINVAL;                                          \
    } while (0)

namespace lqt {
void prolong_project_probes(lqt_ctx*, const lqt_basis*, uint64_t, long long, int, double2*, double2*) {
    throw Error{LQT_EINVAL, "prolongator bases are not implemented in this build"};
}
}  // namespace lqt

extern "C" {

int lqt_basis_prolongator(lqt_ctx* c, const int*, int, int, double, int, const lqt_solver_opts*, lqt_basis**) {
    LQT_PENDING(c);
}
int lqt_precond_set(lqt_ctx* c, const void*, size_t) { LQT_PENDING(c); }
int lqt_precond_get(lqt_ctx* c, void*, size_t) { LQT_PENDING(c); }
int lqt_precond_apply(lqt_ctx* c, const double*, double*, int) { LQT_PENDING(c); }
int lqt_precond_train(lqt_ctx* c, int, uint64_t, const lqt_train_opts*, double*) { LQT_PENDING(c); }
int lqt_restrict(lqt_ctx* c, const lqt_basis*, const double*, double*, int) { LQT_PENDING(c); }
int lqt_prolong(lqt_ctx* c, const lqt_basis*, const double*, double*, int) { LQT_PENDING(c); }
int lqt_prolongator_get(const lqt_basis*, double*, long long*) { return LQT_EINVAL; }
int lqt_basis_prolongator_from(lqt_ctx* c, const int*, int, const double*, lqt_basis**) { LQT_PENDING(c); }

}  // extern "C"

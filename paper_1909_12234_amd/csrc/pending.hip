// Entry points whose implementation is not in this build yet: they fail with LQT_EINVAL
// and say so, so the exported C-ABI is complete and callers get a clear error.
#include "lqt_internal.h"

#define LQT_PENDING(c)                                                                             \
    do {                                                                                           \
        if (c) ((lqt_ctx*)(c))->err = std::string(__func__) + " is not implemented in this build"; \
        return LQT_EINVAL;                                                                         \
    } while (0)

extern "C" {

int lqt_precond_set(lqt_ctx* c, const void*, size_t) { LQT_PENDING(c); }
int lqt_precond_get(lqt_ctx* c, void*, size_t) { LQT_PENDING(c); }
int lqt_precond_apply(lqt_ctx* c, const double*, double*, int) { LQT_PENDING(c); }
int lqt_precond_train(lqt_ctx* c, int, uint64_t, const lqt_train_opts*, double*) { LQT_PENDING(c); }

}  // extern "C"

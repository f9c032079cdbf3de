// Stall detection of restarted solves and the chain of more robust solver settings that a
// stalled system falls back to (host code only).
//
// A restarted solve is assessed on its FP64 true residuals (the only residuals that decide
// convergence).  A system has stalled when
//   - a cycle took no step at all: an s-step cycle whose Gram matrix kept fewer than two
//     columns (the start vector is an eigenvector of A, or 16-bit storage overflowed); the
//     same cycle would repeat unchanged, so this is final; or
//   - `window` FP64 residuals in a row did not fall at least 0.1 % below the smallest one
//     formed before them (restarted GMRES stagnating, or a preconditioner that no longer
//     helps).
// The fallback chain drops, one at a time and in this order, what can make a solve stall:
// the learned preconditioner, the s-step cycles, 16-bit storage (to FP32) and reduced
// storage altogether (to FP64, plain restarted GMRES).  A stalled system restarts from its
// current solution at the next setting that differs from the one it stalled with.
#pragma once

#include <cmath>

namespace lqt {

struct StallWatch {
    int window = 2;     // FP64 residuals without a decrease that count as a stall
    double best = -1;   // smallest FP64 residual norm so far (-1: none formed yet)
    int flat = 0;       // FP64 residuals in a row without a 0.1 % decrease below `best`
    bool zero = false;  // the last cycle took no step

    // record the steps of a finished cycle
    void cycle(int steps) { zero = steps <= 0; }
    // record a newly formed FP64 residual norm rr; true if the system has stalled
    bool formed(double rr) {
        if (zero) return true;
        if (!(rr == rr)) return true;  // not finite: nothing to improve on
        if (best < 0 || rr < (1.0 - 1e-3) * best) {
            best = best < 0 ? rr : std::fmin(best, rr);
            flat = 0;
            return false;
        }
        flat++;
        return window > 0 && flat >= window;
    }
};

// Solver settings that the fallback chain changes.
struct ChainCfg {
    int prec;   // storage precision (LQT_F64 .. LQT_BF16: 0 .. 3)
    int net;    // learned preconditioner on
    int sstep;  // s-step cycles on
};

// The next setting of the chain after `c`; false when `c` is already plain FP64 GMRES.
inline bool chain_next(const ChainCfg& c, ChainCfg& out) {
    out = c;
    if (c.net) {
        out.net = 0;
        return true;
    }
    if (c.sstep) {
        out.sstep = 0;
        return true;
    }
    if (c.prec >= 2) {  // FP16 or BF16 storage -> FP32
        out.prec = 1;
        return true;
    }
    if (c.prec == 1) {
        out.prec = 0;
        return true;
    }
    return false;
}

}  // namespace lqt

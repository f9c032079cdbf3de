// Inexact solves A^{-1}_xi (Section 1: stop when ||A y - x|| <= xi ||x||).
//
// Restarted GMRES(m) over a batch of right-hand sides.  Each restart is an FP64 defect
// correction step: r = b - A x is recomputed with the FP64 operator and tested against
// xi ||b||; the following cycle of at most m Arnoldi steps runs on r / ||r|| with links
// and Krylov vectors in the inner storage precision (FP64, FP32, FP16 or BF16) and
// FP32 (FP64 for FP64 storage) arithmetic, and its correction is added to x in FP64.
// With FP64 storage this is plain restarted GMRES(m).  Systems that converge leave the
// batch at the next restart, so the remaining ones stay contiguous.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

#include "blas.h"
#include "krylov.h"
#include "lqt_internal.h"
#include "ptc.h"
#include "twogrid.h"
#include "solver.h"
#include "stall.h"

namespace lqt {

namespace {

struct StateBuf {
    KryState st;
    void carve(DBuf& buf, int ns, int m) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += (bytes + 255) & ~size_t(255);
            return o;
        };
        size_t oH = take(sizeof(double2) * ns * (m + 1) * m), ocs = take(sizeof(double) * ns * m),
               osn = take(sizeof(double2) * ns * m), og = take(sizeof(double2) * ns * (m + 1)),
               osc = take(sizeof(double) * ns * (m + 1)), oal = take(sizeof(double2) * ns * (m + 1)),
               oy = take(sizeof(double2) * ns * (m + 1)), obe = take(sizeof(double2) * ns * (m + 1)),
               ofa = take(sizeof(double) * ns), onu = take(sizeof(double) * ns), oes = take(sizeof(double) * ns),
               ota = take(sizeof(double) * ns), okd = take(sizeof(int) * ns), ofr = take(sizeof(int) * ns);
        buf.ensure(off);
        char* b = (char*)buf.p;
        st.m = m;
        st.H = (double2*)(b + oH);
        st.cs = (double*)(b + ocs);
        st.sn = (double2*)(b + osn);
        st.g = (double2*)(b + og);
        st.sc = (double*)(b + osc);
        st.alpha = (double2*)(b + oal);
        st.y = (double2*)(b + oy);
        st.beta = (double2*)(b + obe);
        st.fac = (double*)(b + ofa);
        st.nu = (double*)(b + onu);
        st.est = (double*)(b + oes);
        st.target = (double*)(b + ota);
        st.kdim = (int*)(b + okd);
        st.frozen = (int*)(b + ofr);
    }
};

// One Arnoldi orthogonalisation: CGS (or CGS2) dot and update passes.  Algorithmic bytes:
// the dot pass reads j+2 vectors, the update pass reads j+2 and writes one (per slot).
template <typename S>
void kry_step_orth(lqt_ctx* c, void* basis, long long vstride, int j, int na, const KryState& st, bool cgs2,
                   double2* part, double* partn) {
    const double vb = 24.0 * c->g.V * (sizeof(S) / 2) * na;  // bytes of one vector per slot set
    const int nsb = kry_blocks<S>(c);
    for (int pass = 0; pass < (cgs2 ? 2 : 1); pass++) {
        c->timer.begin(c->stream, KT_DOTS);
        kry_dots<S>(c, basis, vstride, j, na, part);
        c->timer.end(c->stream, vb * (j + 2));
        c->timer.begin(c->stream, KT_KRYLOV);
        kry_finish(c, part, nsb, j, na, st, pass);
        c->timer.end(c->stream);
        const int last = (pass == (cgs2 ? 1 : 0));
        c->timer.begin(c->stream, KT_UPDATE);
        kry_update<S>(c, basis, vstride, j, na, st, last, partn);
        c->timer.end(c->stream, vb * (j + 3));
    }
    c->timer.begin(c->stream, KT_KRYLOV);
    kry_norm_givens(c, partn, nsb, j, na, st);
    c->timer.end(c->stream);
}

// Solve nb systems b[0..nb) -> x[0..nb) (device layout FP64, contiguous), from x = 0 or, with
// warm, from the x given.  stalled (host, nb flags, may be null): systems that stalled (see
// stall.h) are set to 1 there and left for the caller's fallback instead of being counted as
// failed; without it only a cycle that took no step ends a system (as failed), and the
// others run until they converge or reach maxit.
template <typename S>
int solve_batch(lqt_ctx* c, int prec, const double2* b, double2* x, int nb, double xi, const SolveOpts& o,
                lqt_solve_stats* stats, bool warm = false, int* stalled = nullptr) {
    const long long n = 12LL * c->g.V;
    const int m = o.restart;
    const size_t eb = sizeof(S);
    const int nsb = std::max(kry_blocks<S>(c), (c->g.V + 255) / 256);  // partial sums per slot

    DBuf& basisb = c->scratch[0];
    DBuf& rb = c->scratch[1];
    DBuf& stb = c->scratch[2];
    DBuf& partb = c->scratch[3];
    DBuf& partnb = c->scratch[4];
    basisb.ensure((size_t)(m + 1) * nb * n * eb);
    // flexible GMRES: z_j = M v_j is kept for the solution update (right preconditioning)
    DBuf& zb = c->scratch[12];
    const bool flex = o.use_net || o.twogrid;
    if (flex) zb.ensure((size_t)m * nb * n * eb);
    rb.ensure((size_t)nb * n * sizeof(double2) + 4 * 256 * (size_t)nb);
    StateBuf sb;
    sb.carve(stb, nb, m);
    partb.ensure(std::max(sizeof(double2) * (size_t)nb * nsb * (m + 2),
                          sizeof(double) * (size_t)nb * kry_carry_blocks<S>(c)));
    const int nlat = c->g.lat.nlat;
    const bool multi = nlat > 1;  // several lattices: every lattice block must meet xi
    // s-step basis k_{i+1} = sigma (A - theta) k_i: theta = 4 + m centres the spectrum of A
    // (A - theta is the hopping term), sigma = 1/2 keeps the vectors' scale near one
    double theta = 0;
    for (int l = 0; l < nlat; l++) theta += c->g.lat.diag[l] / nlat;
    const double sigma = 0.5;
    if (o.sstep) c->scratch[13].ensure(sizeof(double) * (size_t)nb * 64 * (m + 1) * (m + 2));  // before any capture
    partnb.ensure(sizeof(double) * (size_t)nb * nsb + sizeof(double) * 2 * nb + sizeof(int) * 2 * nb +
                  sizeof(double) * nb + sizeof(double) * (size_t)nb * nlat + sizeof(double) * nb + 1024);
    // s-step cycles on one lattice carry the residual in the basis between FP64 residuals
    const bool carry = o.sstep && o.reliable > 0 && !multi;

    double2* r = rb.as<double2>();
    char* extra = (char*)partnb.p + sizeof(double) * (size_t)nb * nsb;
    double* rn2 = (double*)extra;
    double* bn2 = rn2 + nb;
    int* act_d = (int*)(bn2 + nb);
    int* src_d = act_d + nb;
    double* tgt_d = (double*)(((uintptr_t)(src_d + nb) + 7) & ~uintptr_t(7));
    double* rn2l = tgt_d + nb;  // [slot][lattice]
    double* rn2c = rn2l + (size_t)nb * nlat;  // |carried residual|^2 per slot
    double* partn = partnb.as<double>();
    double2* part = partb.as<double2>();
    void* basis = basisb.p;

    c->pinned.ensure(sizeof(double) * (5 + (size_t)nlat) * nb + 64);
    double* h_rn2 = c->pinned.as<double>();
    int* h_flags = (int*)(h_rn2 + nb);
    double* h_rn2l = h_rn2 + 2 * (size_t)nb;
    double* h_rn2c = h_rn2l + (size_t)nlat * nb;

    std::vector<double> bnorm(nb);
    c->timer.begin(c->stream, KT_KRYLOV);
    norm2_fields(c, b, nb, bn2);
    if (!warm) LQT_HIP(hipMemsetAsync(x, 0, sizeof(double2) * (size_t)nb * n, c->stream));
    c->timer.end(c->stream);
    LQT_HIP(hipMemcpyAsync(h_rn2, bn2, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < nb; i++) bnorm[i] = std::sqrt(h_rn2[i]);
    std::vector<double> bnl;  // |b| per (system, lattice)
    if (multi) {
        norm2_lattices(c, b, nb, rn2l);
        bnl.resize((size_t)nb * nlat);
        LQT_HIP(hipMemcpyAsync(bnl.data(), rn2l, sizeof(double) * bnl.size(), hipMemcpyDeviceToHost, c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        for (double& v : bnl) v = std::sqrt(v);
    }

    // graph-captured cycles per active count, destroyed when the batch is done
    struct Graphs {
        std::map<int, hipGraphExec_t> m;
        hipGraphExec_t& operator[](int k) { return m[k]; }
        ~Graphs() {
            for (auto& kv : m)
                if (kv.second) (void)hipGraphExecDestroy(kv.second);
        }
    } graphs;
    std::vector<int> act(nb), its(nb, 0), cyc(nb, 0), done(nb, 0);
    std::vector<double> rel(nb, 1.0), rlast(nb, 0.0);
    std::vector<StallWatch> watch(nb);
    for (int i = 0; i < nb; i++) {
        act[i] = i;
        watch[i].window = stalled ? o.stall_window : 0;  // no fallback: only zero-step cycles end a system
    }
    int nfail = 0;
    bool carried = false;  // the basis start vectors hold the residuals carried from the last cycle

    while (!act.empty()) {
        const int na = (int)act.size();
        // A cycle may start from the carried residual unless some system's carried residual
        // meets the tolerance, fell below `reliable` times its last FP64 residual, is not
        // finite or the step cap is reached: then every active system gets its FP64 residual.
        bool from_carry = carried;
        for (int k = 0; k < na && from_carry; k++) {
            const int i = act[k];
            const double rr = std::sqrt(h_rn2c[k]);
            if (!(rr == rr) || rr <= xi * bnorm[i] || rr <= o.reliable * rlast[i] || its[i] >= o.maxit)
                from_carry = false;
        }
        if (from_carry) {
            std::vector<double> tgt(na);
            for (int k = 0; k < na; k++) {
                const int i = act[k];
                const double rr = std::sqrt(h_rn2c[k]);
                cyc[i]++;
                rel[i] = bnorm[i] > 0 ? rr / bnorm[i] : 0.0;
                tgt[k] = std::max(xi * bnorm[i], o.inner_tol * rr);
            }
            LQT_HIP(hipMemcpyAsync(tgt_d, tgt.data(), sizeof(double) * na, hipMemcpyHostToDevice, c->stream));
            c->timer.begin(c->stream, KT_KRYLOV);
            kry_start_state_carry(c, sb.st, tgt_d, na);
            c->timer.end(c->stream);
        }
        std::vector<int> nact;
        if (from_carry) {
            nact = act;
        } else {
            LQT_HIP(hipMemcpyAsync(act_d, act.data(), sizeof(int) * na, hipMemcpyHostToDevice, c->stream));
            residual64(c, b, x, r, rn2, na, act_d, multi ? rn2l : nullptr);
            LQT_HIP(hipMemcpyAsync(h_rn2, rn2, sizeof(double) * na, hipMemcpyDeviceToHost, c->stream));
            if (multi)
                LQT_HIP(hipMemcpyAsync(h_rn2l, rn2l, sizeof(double) * na * nlat, hipMemcpyDeviceToHost, c->stream));
            LQT_HIP(hipStreamSynchronize(c->stream));
            std::vector<int> src;
            std::vector<double> tgt;
            for (int k = 0; k < na; k++) {
                const int i = act[k];
                cyc[i]++;
                double rr = std::sqrt(h_rn2[k]);
                rlast[i] = rr;
                rel[i] = bnorm[i] > 0 ? rr / bnorm[i] : 0.0;
                double bmin = bnorm[i];  // the cycle target must serve the smallest lattice block
                if (multi) {
                    double worst = 0;
                    for (int l = 0; l < nlat; l++) {
                        const double bl = bnl[(size_t)i * nlat + l], rl = std::sqrt(h_rn2l[(size_t)k * nlat + l]);
                        if (bl > 0) {
                            worst = std::max(worst, rl / bl);
                            bmin = std::min(bmin, bl);
                        } else if (!(rl == rl)) {
                            worst = rl;
                        }
                    }
                    rel[i] = (rr == rr) ? worst : rr;
                }
                if (!(rel[i] == rel[i])) {  // not finite: the fallback restarts it from zero
                    done[i] = 1;
                    if (stalled)
                        stalled[i] = 2;
                    else
                        nfail++;
                    continue;
                }
                if (rel[i] <= xi) {
                    done[i] = 1;
                    continue;
                }
                if (its[i] >= o.maxit) {
                    done[i] = 1;
                    nfail++;
                    continue;
                }
                if (watch[i].formed(rr)) {  // stalled: hand over to the fallback, else failed
                    done[i] = 1;
                    if (stalled)
                        stalled[i] = 1;
                    else
                        nfail++;
                    continue;
                }
                nact.push_back(i);
                src.push_back(k);
                tgt.push_back(std::max(xi * bmin, o.inner_tol * rr));
            }
            if (nact.empty()) break;
            const int nn0 = (int)nact.size();
            // new active list; src maps new slot -> slot of r
            LQT_HIP(hipMemcpyAsync(act_d, nact.data(), sizeof(int) * nn0, hipMemcpyHostToDevice, c->stream));
            LQT_HIP(hipMemcpyAsync(src_d, src.data(), sizeof(int) * nn0, hipMemcpyHostToDevice, c->stream));
            LQT_HIP(hipMemcpyAsync(tgt_d, tgt.data(), sizeof(double) * nn0, hipMemcpyHostToDevice, c->stream));
            c->timer.begin(c->stream, KT_KRYLOV);
            kry_start_state(c, sb.st, src_d, rn2, tgt_d, nn0);
            kry_start<S>(c, basis, r, src_d, rn2, nn0);
            c->timer.end(c->stream);
        }
        const int nn = (int)nact.size();
        if (o.verbose && (cyc[nact[0]] % 16) == 0) {
            double mx = 0;
            for (int i : nact) mx = std::max(mx, rel[i]);
            fprintf(stderr, "[lqtrace] solve: %d of %d systems active, cycle %d, max relres %.3e%s\n", nn, nb,
                    cyc[nact[0]], mx, from_carry ? " (carried)" : "");
            fflush(stderr);
        }
        const long long vstride = (long long)nn * n;
        // one Arnoldi step: (preconditioner,) operator, Gram-Schmidt and the Givens update;
        // s-step cycles: the operator step k_{j+1} = sigma (A - theta) k_j only
        auto step = [&](int j) {
            const void* vj = (const char*)basis + (size_t)j * vstride * eb;
            void* vj1 = (char*)basis + (size_t)(j + 1) * vstride * eb;
            if (o.sstep) {
                dslash(c, prec, LQT_A, vj, vj1, nn, n, n, theta, sigma);
                return;
            }
            const void* aj = vj;
            if (flex) {
                void* zj = (char*)zb.p + (size_t)j * vstride * eb;
                if (o.use_net)
                    ptc_apply<S>(c, (const S*)vj, (S*)zj, nn);
                else
                    twogrid_apply<S>(c, (const S*)vj, (S*)zj, nn, o);
                aj = zj;
            }
            dslash(c, prec, LQT_A, aj, vj1, nn, n, n);
            kry_step_orth<S>(c, basis, vstride, j, nn, sb.st, o.cgs2 != 0, part, partn);
        };
        auto finish = [&]() {
            if (o.sstep)
                sstep_finish<S>(c, basis, vstride, m, nn, sb.st, theta, sigma, c->scratch[13]);
            c->timer.begin(c->stream, KT_KRYLOV);
            if (!o.sstep) kry_backsolve(c, nn, sb.st);
            if (carry)
                kry_sstep_carry<S>(c, x, act_d, basis, vstride, nn, sb.st, theta, sigma, (double*)part, rn2c);
            else
                kry_xupdate<S>(c, x, act_d, flex ? zb.p : basis, vstride, nn, sb.st);
            c->timer.end(c->stream);
        };
        if (o.graph) {
            // the cycle of nn systems as one graph: captured on a private stream (the
            // context stream may be the null stream), replayed on the context stream
            hipGraphExec_t& ex = graphs[nn];
            if (!ex) {
                if (!c->capture_stream) LQT_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
                if (o.use_net) c->net.act.ensure(sizeof(float2) * (size_t)nn * 24 * c->g.V * 2);
                const hipStream_t s0 = c->stream;
                const bool timing = c->timer.on;
                c->timer.on = false;
                c->stream = c->capture_stream;
                hipGraph_t gr = nullptr;
                hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    try {
                        for (int j = 0; j < m; j++) step(j);
                        finish();
                    } catch (...) {
                        (void)hipStreamEndCapture(c->stream, &gr);
                        if (gr) (void)hipGraphDestroy(gr);
                        c->stream = s0;
                        c->timer.on = timing;
                        throw;
                    }
                    e = hipStreamEndCapture(c->stream, &gr);
                }
                c->stream = s0;
                c->timer.on = timing;
                LQT_HIP(e);
                e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                LQT_HIP(e);
            }
            c->timer.begin(c->stream, KT_GRAPH);
            LQT_HIP(hipGraphLaunch(ex, c->stream));
            c->timer.end(c->stream, 0);
        } else {
            for (int j = 0; j < m; j++) {
                step(j);
                if (j + 1 < m && !o.sstep) {  // stop the cycle once every system's cycle has ended
                    LQT_HIP(hipMemcpyAsync(h_flags, sb.st.frozen, sizeof(int) * nn, hipMemcpyDeviceToHost,
                                           c->stream));
                    LQT_HIP(hipStreamSynchronize(c->stream));
                    bool all = true;
                    for (int k = 0; k < nn; k++) all = all && h_flags[k];
                    if (all) break;
                }
            }
            finish();
        }
        LQT_HIP(hipMemcpyAsync(h_flags, sb.st.kdim, sizeof(int) * nn, hipMemcpyDeviceToHost, c->stream));
        if (carry) LQT_HIP(hipMemcpyAsync(h_rn2c, rn2c, sizeof(double) * nn, hipMemcpyDeviceToHost, c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        // a cycle that took no step would repeat unchanged: its system gets an FP64 residual
        // next, where the stall watch ends it; at least one step is charged against maxit
        bool any_zero = false;
        for (int k = 0; k < nn; k++) {
            its[nact[k]] += std::max(h_flags[k], 1);
            watch[nact[k]].cycle(h_flags[k]);
            any_zero = any_zero || h_flags[k] <= 0;
        }
        act = nact;
        carried = carry && !any_zero;
    }
    if (stats)
        for (int i = 0; i < nb; i++) {
            stats[i].converged = (rel[i] <= xi) ? 1 : 0;
            stats[i].iters = its[i];
            stats[i].cycles = cyc[i];
            stats[i].relres = rel[i];
        }
    return nfail;
}

}  // namespace

// Solve with storage type chosen by prec (see solve_batch).
static int solve_dispatch(lqt_ctx* c, int prec, const double2* b, double2* x, int nb, double xi, const SolveOpts& o,
                          lqt_solve_stats* stats, bool warm, int* stalled) {
    switch (prec) {
        case LQT_F64: return solve_batch<double2>(c, prec, b, x, nb, xi, o, stats, warm, stalled);
        case LQT_F32: return solve_batch<float2>(c, prec, b, x, nb, xi, o, stats, warm, stalled);
        case LQT_F16: return solve_batch<h2>(c, prec, b, x, nb, xi, o, stats, warm, stalled);
        default: return solve_batch<b2>(c, prec, b, x, nb, xi, o, stats, warm, stalled);
    }
}

// The fallback chain for the systems of one batch flagged in `stalled` (1: restart from the
// current x, 2: from zero): each level of the chain (stall.h) solves them again, gathered
// into a contiguous batch, and scatters the solutions back; steps and cycles add up in the
// statistics, whose `fallback` field gets the level.  maxit applies to each level.
// Returns the systems that still missed the tolerance.
static int run_fallback(lqt_ctx* c, const double2* b, double2* x, int nb, double xi, const SolveOpts& o0,
                        lqt_solve_stats* stats, std::vector<int>& stalled) {
    const long long n = 12LL * c->g.V;
    const size_t fb = sizeof(double2) * (size_t)n;
    std::vector<int> idx, how;
    for (int i = 0; i < nb; i++)
        if (stalled[i]) {
            idx.push_back(i);
            how.push_back(stalled[i]);
        }
    ChainCfg cur{o0.prec, o0.use_net || o0.twogrid, o0.sstep};
    int level = 0, nfail = 0;
    while (!idx.empty()) {
        ChainCfg nx;
        if (!chain_next(cur, nx)) {  // plain FP64 GMRES stalled as well
            nfail += (int)idx.size();
            break;
        }
        cur = nx;
        level++;
        SolveOpts o = o0;
        o.prec = cur.prec;
        o.use_net = cur.net ? o0.use_net : 0;
        o.twogrid = cur.net ? o0.twogrid : 0;
        o.sstep = cur.sstep;
        const int ns = (int)idx.size();
        if (o0.verbose) {
            fprintf(stderr, "[lqtrace] solve: %d stalled system(s) continue at fallback level %d (storage %d%s%s)\n",
                    ns, level, o.prec, o.use_net ? ", net" : (o.twogrid ? ", two-grid" : ""), o.sstep ? ", s-step" : "");
            fflush(stderr);
        }
        DBuf bs, xs;
        bs.ensure(fb * ns);
        xs.ensure(fb * ns);
        for (int k = 0; k < ns; k++) {
            LQT_HIP(hipMemcpyAsync((char*)bs.p + fb * k, b + (size_t)idx[k] * n, fb, hipMemcpyDeviceToDevice,
                                   c->stream));
            if (how[k] == 2)
                LQT_HIP(hipMemsetAsync((char*)xs.p + fb * k, 0, fb, c->stream));
            else
                LQT_HIP(hipMemcpyAsync((char*)xs.p + fb * k, x + (size_t)idx[k] * n, fb, hipMemcpyDeviceToDevice,
                                       c->stream));
        }
        std::vector<lqt_solve_stats> sub(ns);
        std::vector<int> st2(ns, 0);
        nfail += solve_dispatch(c, o.prec, bs.as<double2>(), xs.as<double2>(), ns, xi, o, sub.data(), true,
                                st2.data());
        for (int k = 0; k < ns; k++)
            LQT_HIP(hipMemcpyAsync(x + (size_t)idx[k] * n, (char*)xs.p + fb * k, fb, hipMemcpyDeviceToDevice,
                                   c->stream));
        LQT_HIP(hipStreamSynchronize(c->stream));
        std::vector<int> nidx, nhow;
        for (int k = 0; k < ns; k++) {
            if (stats) {
                lqt_solve_stats& t = stats[idx[k]];
                t.converged = sub[k].converged;
                t.iters += sub[k].iters;
                t.cycles += sub[k].cycles;
                t.relres = sub[k].relres;
                t.fallback = level;
            }
            if (st2[k]) {
                nidx.push_back(idx[k]);
                nhow.push_back(st2[k]);
            }
        }
        idx.swap(nidx);
        how.swap(nhow);
    }
    return nfail;
}

SolveOpts make_opts(const lqt_solver_opts* u) {
    SolveOpts o;
    if (u) {
        o.prec = u->inner_prec;
        o.restart = u->restart > 0 ? u->restart : 32;
        o.maxit = u->maxit > 0 ? u->maxit : 100000;
        o.use_net = u->use_net;
        o.max_batch = u->max_batch;
        o.cgs2 = u->cgs2;
        o.inner_tol = u->inner_tol > 0 ? u->inner_tol : 0.0;
        o.verbose = u->verbose;
        o.outer_maxit = u->outer_maxit > 0 ? u->outer_maxit : 200;
        o.graph = u->graph;
        o.sstep = u->sstep;
        o.reliable = u->reliable < 0 ? 0.0 : (u->reliable > 0 ? u->reliable : 0.1);
        o.fallback = u->fallback;
        o.stall_window = u->stall_window > 0 ? u->stall_window : 2;
        o.eig_degree = u->eig_degree > 0 ? u->eig_degree : 128;
        o.eig_xi = u->eig_xi > 0 ? u->eig_xi : 0.0;
        o.twogrid = u->twogrid;
        o.tg_smooth = u->tg_smooth > 0 ? u->tg_smooth : (u->tg_smooth < 0 ? 0 : 4);
        o.tg_coarse_tol = u->tg_coarse_tol > 0 ? u->tg_coarse_tol : 0.1;
        o.tg_coarse_maxit = u->tg_coarse_maxit > 0 ? u->tg_coarse_maxit : 32;
    }
    return o;
}

int solve_fields(lqt_ctx* c, const double2* b, double2* x, int nrhs, double xi, const SolveOpts& o,
                 lqt_solve_stats* stats) {
    LQT_CHECK(o.restart >= 1 && o.restart <= KRY_MAXM, LQT_EINVAL, "restart must be in 1..64");
    LQT_CHECK(o.prec >= LQT_F64 && o.prec <= LQT_BF16, LQT_EINVAL, "bad inner precision");
    LQT_CHECK(xi > 0, LQT_EINVAL, "tolerance must be positive");
    LQT_CHECK(!o.use_net || c->net.set, LQT_ESTATE, "use_net requires preconditioner weights (lqt_precond_set/train)");
    LQT_CHECK(!o.use_net || c->g.lat.nlat == 1, LQT_EINVAL, "the network preconditioner serves single-lattice contexts");
    LQT_CHECK(!(o.use_net && o.twogrid), LQT_EINVAL, "use_net and twogrid are exclusive");
    LQT_CHECK(!o.twogrid || c->tg, LQT_ESTATE, "twogrid requires a prolongator (lqt_precond_twogrid)");
    LQT_CHECK(!o.twogrid || !o.graph, LQT_EINVAL, "the two-grid preconditioner cannot run inside a captured graph");
    LQT_CHECK(!o.sstep || (!o.use_net && !o.twogrid && o.restart <= (storage_bytes(o.prec) == 4 ? 15 : 8)), LQT_EINVAL,
              "s-step cycles need restart <= 15 (16-bit storage) or <= 8, and no network preconditioner");
    LQT_CHECK(o.reliable >= 0 && o.reliable < 1, LQT_EINVAL, "reliable must be below 1");
    const long long n = 12LL * c->g.V;
    // batch size: caller cap, else what fits in 70% of free device memory
    size_t fr = 0, tot = 0;
    LQT_HIP(hipMemGetInfo(&fr, &tot));
    size_t per = (size_t)(o.restart + 1) * n * storage_bytes(o.prec) + (size_t)n * 16 * 2 +
                 (size_t)((c->g.V + 255) / 256) * (o.restart + 2) * 16;
    if (o.use_net) per += (size_t)o.restart * n * storage_bytes(o.prec) + (size_t)c->g.V * 24 * 8 * 2;
    if (o.twogrid) per += (size_t)o.restart * n * storage_bytes(o.prec) + (size_t)n * 16 * 4;
    size_t have = (size_t)(0.7 * (double)(fr + c->scratch[0].n + c->scratch[1].n + c->scratch[3].n +
                                          c->scratch[12].n + c->net.act.n));
    int fit = (int)std::max<size_t>(1, have / per);
    int batch = o.max_batch > 0 ? o.max_batch : nrhs;
    batch = std::min(batch, fit);
    int nfail = 0;
    for (int b0 = 0; b0 < nrhs; b0 += batch) {
        int nb = std::min(batch, nrhs - b0);
        const double2* bb = b + (size_t)b0 * n;
        double2* xx = x + (size_t)b0 * n;
        lqt_solve_stats* ss = stats ? stats + b0 : nullptr;
        if (ss)
            for (int i = 0; i < nb; i++) ss[i].fallback = 0;
        std::vector<int> stalled(o.fallback ? nb : 0, 0);
        nfail += solve_dispatch(c, o.prec, bb, xx, nb, xi, o, ss, false, o.fallback ? stalled.data() : nullptr);
        if (o.fallback) nfail += run_fallback(c, bb, xx, nb, xi, o, ss, stalled);
    }
    return nfail;
}

}  // namespace lqt

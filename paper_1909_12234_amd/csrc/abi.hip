// C-ABI entry points of lqtrace.  Every call catches library errors and converts them to
// the LQT_E* codes; the message stays in the context.
#include <cmath>
#include <cstring>
#include <new>

#include "blas.h"
#include "devla.h"
#include "lqt_internal.h"
#include "solver.h"

using lqt::DBuf;
using lqt::Error;

namespace {

template <typename F>
int guard(lqt_ctx* c, F&& f) {
    try {
        f();
        return LQT_OK;
    } catch (const Error& e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return LQT_ENOMEM;
    } catch (...) {
        if (c) c->err = "unexpected exception";
        return LQT_EINVAL;
    }
}

void need_gauge(lqt_ctx* c) { LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)"); }

}  // namespace

extern "C" {

int lqt_create(lqt_ctx** ctx, const int dims[4], double mass, int t_antiperiodic, void* hip_stream) {
    if (!ctx) return LQT_EINVAL;
    *ctx = nullptr;
    if (!dims) return LQT_EINVAL;
    long long V = 1;
    for (int i = 0; i < 4; i++) {
        if (dims[i] < 2) return LQT_EINVAL;
        V *= dims[i];
    }
    // every FP64 field of one right-hand side stays below 4 GiB (32-bit byte offsets in the kernels)
    if (V > (1LL << 32) / (12 * 16) - 256 || !std::isfinite(mass)) return LQT_EINVAL;
    lqt_ctx* c = new (std::nothrow) lqt_ctx();
    if (!c) return LQT_ENOMEM;
    for (int i = 0; i < 4; i++) c->g.L[i] = dims[i];
    c->g.V = (int)V;
    c->g.lat.nlat = 1;
    for (int i = 0; i < 4; i++) c->g.lat.L[0][i] = dims[i];
    c->g.lat.off[0] = 0;
    c->g.lat.off[1] = (int)V;
    c->g.lat.coff[0] = 0;
    c->g.lat.coff[1] = (int)V;
    c->g.lat.diag[0] = 4.0 + mass;
    c->g.canon_sites = V;
    c->N = 12 * V;
    c->mass = mass;
    c->antiperiodic = t_antiperiodic ? 1 : 0;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LQT_EHIP;
    }
    try {
        lqt::static_scratch_init(c->device);  // device address of lqt_gram_noalloc's workspace
    } catch (const lqt::Error& e) {
        delete c;
        return e.code;
    }
    c->timer.init();
    *ctx = c;
    return LQT_OK;
}

int lqt_create_multi(lqt_ctx** ctx, int nlat, const int* dims, const double* masses, int t_antiperiodic,
                     void* hip_stream) {
    if (!ctx) return LQT_EINVAL;
    *ctx = nullptr;
    if (nlat < 1 || nlat > lqt::LQT_MAXLAT || !dims || !masses) return LQT_EINVAL;
    lqt::LatTab t{};
    t.nlat = nlat;
    long long off = 0, coff = 0;
    for (int k = 0; k < nlat; k++) {
        long long Vk = 1;
        for (int i = 0; i < 4; i++) {
            if (dims[4 * k + i] < 2) return LQT_EINVAL;
            t.L[k][i] = dims[4 * k + i];
            Vk *= dims[4 * k + i];
        }
        if (!std::isfinite(masses[k])) return LQT_EINVAL;
        t.off[k] = (int)off;
        t.coff[k] = (int)coff;
        t.diag[k] = 4.0 + masses[k];
        off += (Vk + 255) / 256 * 256;  // each lattice starts on a 256-site boundary
        coff += Vk;
        if (off > (1LL << 32) / (12 * 16) - 256) return LQT_EINVAL;
    }
    t.off[nlat] = (int)off;
    t.coff[nlat] = (int)coff;
    int rc = lqt_create(ctx, dims, masses[0], t_antiperiodic, hip_stream);
    if (rc != LQT_OK) return rc;
    lqt_ctx* c = *ctx;
    c->g.lat = t;
    c->g.V = (int)off;
    c->g.canon_sites = coff;
    c->N = 12 * off;
    return LQT_OK;
}

void lqt_destroy(lqt_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    c->timer.destroy();
    lqt::blas_release(c);
    delete c;
}

const char* lqt_last_error(const lqt_ctx* c) { return c ? c->err.c_str() : "null context"; }

int lqt_set_gauge(lqt_ctx* c, const double* links, int on_device) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(links, LQT_EINVAL, "links is null");
        double eu = 0, ed = 0;
        lqt::gauge_upload(c, links, on_device, &eu, &ed);
        c->have_gauge = false;
        LQT_CHECK(eu < 1e299 && ed < 1e299, LQT_ENAN, "gauge field holds NaN or Inf");
        LQT_CHECK(eu <= 1e-10 && ed <= 1e-10, LQT_ENOTUNITARY,
                  "gauge link not special unitary: max|U^+U-1| = " + std::to_string(eu) +
                      ", max|det U - 1| = " + std::to_string(ed));
        c->have_gauge = true;
        c->sigma_max = 0;
    });
}

int lqt_set_mass(lqt_ctx* c, double mass) {
    if (!c) return LQT_EINVAL;
    if (!std::isfinite(mass)) return LQT_EINVAL;
    c->mass = mass;
    for (int k = 0; k < c->g.lat.nlat; k++) c->g.lat.diag[k] = 4.0 + mass;
    c->sigma_max = 0;
    return LQT_OK;
}

int lqt_apply(lqt_ctx* c, int op, int prec, const void* in, void* out, int nrhs) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(op >= LQT_A && op <= LQT_G5_A, LQT_EINVAL, "bad operator");
        LQT_CHECK(prec >= LQT_F64 && prec <= LQT_BF16, LQT_EINVAL, "bad precision");
        LQT_CHECK(nrhs >= 0, LQT_EINVAL, "nrhs < 0");
        if (nrhs == 0) return;
        LQT_CHECK(in && out, LQT_EINVAL, "null field pointer");
        need_gauge(c);
        const long long n = 12LL * c->g.V;
        const size_t eb = lqt::storage_bytes(prec);
        c->scratch[5].ensure((size_t)n * nrhs * eb);
        c->scratch[6].ensure((size_t)n * nrhs * eb);
        void* a = c->scratch[5].p;
        void* b = c->scratch[6].p;
        switch (prec) {
            case LQT_F64: lqt::to_device_layout(c, (const double2*)in, (double2*)a, nrhs); break;
            case LQT_F32: lqt::convert_in_c64<float2>(c, (const float2*)in, (float2*)a, nrhs); break;
            case LQT_F16: lqt::convert_in_c64<lqt::h2>(c, (const float2*)in, (lqt::h2*)a, nrhs); break;
            default: lqt::convert_in_c64<lqt::b2>(c, (const float2*)in, (lqt::b2*)a, nrhs); break;
        }
        lqt::dslash(c, prec, op, a, b, nrhs, n, n);
        switch (prec) {
            case LQT_F64: lqt::from_device_layout(c, (const double2*)b, (double2*)out, nrhs); break;
            case LQT_F32: lqt::convert_out_c64<float2>(c, (const float2*)b, (float2*)out, nrhs); break;
            case LQT_F16: lqt::convert_out_c64<lqt::h2>(c, (const lqt::h2*)b, (float2*)out, nrhs); break;
            default: lqt::convert_out_c64<lqt::b2>(c, (const lqt::b2*)b, (float2*)out, nrhs); break;
        }
    });
}

int lqt_solve(lqt_ctx* c, const double* b, double* x, int nrhs, double xi, const lqt_solver_opts* opts,
              lqt_solve_stats* stats) {
    if (!c) return LQT_EINVAL;
    int nfail = 0;
    int rc = guard(c, [&] {
        LQT_CHECK(nrhs >= 0, LQT_EINVAL, "nrhs < 0");
        if (nrhs == 0) return;
        LQT_CHECK(b && x, LQT_EINVAL, "null field pointer");
        LQT_CHECK(xi > 0 && std::isfinite(xi), LQT_EINVAL, "tolerance must be positive");
        need_gauge(c);
        lqt::SolveOpts o = lqt::make_opts(opts);
        LQT_CHECK(!o.use_net || c->net.set, LQT_ESTATE, "use_net without preconditioner weights");
        const long long n = 12LL * c->g.V;
        const long long ncanon = 12LL * c->g.canon_sites;  // the caller's field length
        LQT_CHECK(!lqt::has_nonfinite(c, b, (size_t)(2 * ncanon * nrhs)), LQT_ENAN, "right-hand side holds NaN or Inf");
        DBuf bd, xd;
        bd.ensure(sizeof(double2) * (size_t)n * nrhs);
        xd.ensure(sizeof(double2) * (size_t)n * nrhs);
        lqt::to_device_layout(c, (const double2*)b, bd.as<double2>(), nrhs);
        nfail = lqt::solve_fields(c, bd.as<double2>(), xd.as<double2>(), nrhs, xi, o, stats);
        lqt::from_device_layout(c, xd.as<double2>(), (double2*)x, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
        if (nfail) c->err = std::to_string(nfail) + " of " + std::to_string(nrhs) + " systems missed the tolerance";
    });
    if (rc == LQT_OK && nfail) return LQT_ENOTCONV;
    return rc;
}

int lqt_partition_probes(lqt_ctx* c, uint64_t seed, long long p0, int nvec, int hp_vectors, int dilute, double* out) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(nvec >= 0 && p0 >= 0, LQT_EINVAL, "bad vector range");
        lqt::check_partition(c, hp_vectors, dilute);
        if (nvec == 0) return;
        LQT_CHECK(out, LQT_EINVAL, "null output");
        const long long n = 12LL * c->g.V;
        DBuf t;
        t.ensure(sizeof(double2) * (size_t)n * nvec);
        for (int f0 = 0; f0 < nvec; f0 += 65535) {
            const int cnt = std::min(65535, nvec - f0);
            lqt::partition_probes_gen(c, seed, p0 + f0, cnt, hp_vectors, dilute, t.as<double2>() + (size_t)f0 * n);
        }
        lqt::from_device_layout(c, t.as<double2>(), (double2*)out, nvec);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_probes(lqt_ctx* c, uint64_t seed, long long j0, int nprobes, double* out) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(nprobes >= 0 && j0 >= 0, LQT_EINVAL, "bad probe range");
        if (nprobes == 0) return;
        LQT_CHECK(out, LQT_EINVAL, "null output");
        const long long n = 12LL * c->g.V;
        DBuf t;
        t.ensure(sizeof(double2) * (size_t)n * nprobes);
        lqt::probes_gen(c, seed, j0, nprobes, t.as<double2>());
        lqt::from_device_layout(c, t.as<double2>(), (double2*)out, nprobes);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_tune(lqt_ctx* c, int prec, int nrhs, double* ms, int* tile) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(prec >= LQT_F64 && prec <= LQT_BF16 && nrhs >= 1, LQT_EINVAL, "bad tuning request");
        need_gauge(c);
        lqt::Tuned t;
        double best = lqt::dslash_tune(c, prec, nrhs, &t);
        lqt::residual_tune(c, nrhs);  // the FP64 defect-correction residual for this batch size
        if (ms) *ms = best;
        if (tile) {
            tile[0] = t.rhs_per_thread;
            tile[1] = t.block;
            tile[2] = t.chunk;
            tile[3] = t.kind;
        }
    });
}

int lqt_set_tile(lqt_ctx* c, int prec, int nrhs, const int* tile) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(prec >= LQT_F64 && prec <= LQT_BF16 && nrhs >= 1 && tile, LQT_EINVAL, "bad tiling request");
        lqt::Tuned t{tile[0], tile[1], tile[2]};
        t.kind = tile[3];
        LQT_CHECK(t.block == 64 || t.block == 128 || t.block == 256, LQT_EINVAL, "block must be 64, 128 or 256");
        LQT_CHECK(t.chunk >= 0, LQT_EINVAL, "chunk must be >= 0");
        if (t.kind == 4) {
            LQT_CHECK(prec == LQT_F16 && t.block == 256 && t.rhs_per_thread == 1, LQT_EINVAL,
                      "the streaming kernel takes FP16 storage, 256-thread blocks and one rhs per thread");
        } else if (t.kind == 0 || t.kind == 2 || t.kind == 3) {
            LQT_CHECK(t.rhs_per_thread == 1 || t.rhs_per_thread == 2 || (t.rhs_per_thread == 4 && prec != LQT_F64),
                      LQT_EINVAL, "rhs per thread must be 1, 2 or 4 (1 or 2 for FP64)");
            LQT_CHECK(t.kind == 0 || prec == LQT_F16, LQT_EINVAL, "packed half-precision arithmetic takes FP16 storage");
            LQT_CHECK(t.kind != 3 || t.block == 256, LQT_EINVAL, "the staged-link kernel takes 256-thread blocks");
        } else {
            LQT_CHECK(t.kind == 1 && (prec == LQT_F16 || prec == LQT_BF16), LQT_EINVAL,
                      "the matrix-core kernel takes FP16 or BF16 storage");
            LQT_CHECK(t.rhs_per_thread == 1 || t.rhs_per_thread == 2, LQT_EINVAL, "groups per lane must be 1 or 2");
        }
        c->tuned[lqt::tune_key(prec, nrhs)] = t;
    });
}

int lqt_kernel_times(lqt_ctx* c, double* ms, long long* calls, double* bytes, int mode) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        c->timer.flush();
        for (int i = 0; i < lqt::KT_N; i++) {
            if (ms) ms[i] = c->timer.ms[i];
            if (calls) calls[i] = c->timer.calls[i];
            if (bytes) bytes[i] = c->timer.bytes[i];
        }
        if (mode == 1) c->timer.reset();
        if (mode == 2) {
            c->timer.reset();
            c->timer.on = true;
        }
        if (mode == 3) c->timer.on = false;
    });
}

}  // extern "C"

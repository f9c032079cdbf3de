// Internal declarations of the lqtrace HIP library (gfx950).
//
// Device layouts
//   gauge   [mu][ab][V]        complex<S>; the antiperiodic -1 is folded into U_t on the
//                              last time slice (t = Lt-1), so kernels never test borders
//                              for signs.
//   fields  [rhs][comp][V]     complex<S>, comp = 3*spin + colour (12 per site); every
//                              component of every site is one coalesced lane load.
//   FP64 canonical fields at the boundary are converted to/from this layout on entry.
// Storage types S: double2, float2, h2 (two FP16), b2 (two BF16).  Arithmetic is FP64 for
// double2 and FP32 for the others.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/lqtrace.h"

namespace lqt {

// ------------------------------------------------------------------ storage types
struct h2 {
    __half x, y;
};
struct b2 {
    uint16_t x, y;
};

template <typename S>
struct acc_of {
    using type = float;
};
template <>
struct acc_of<double2> {
    using type = double;
};

template <typename C>
struct cplx2;
template <>
struct cplx2<float> {
    using type = float2;
};
template <>
struct cplx2<double> {
    using type = double2;
};

__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

template <typename S>
struct io;
template <>
struct io<double2> {
    __device__ __forceinline__ static double2 ld(const double2* p) { return *p; }
    __device__ __forceinline__ static void st(double2* p, double2 v) { *p = v; }
};
template <>
struct io<float2> {
    __device__ __forceinline__ static float2 ld(const float2* p) { return *p; }
    __device__ __forceinline__ static void st(float2* p, float2 v) { *p = v; }
};
template <>
struct io<h2> {
    __device__ __forceinline__ static float2 ld(const h2* p) {
        h2 v = *p;
        return make_float2(__half2float(v.x), __half2float(v.y));
    }
    __device__ __forceinline__ static void st(h2* p, float2 v) {
        h2 o;
        o.x = __float2half_rn(v.x);
        o.y = __float2half_rn(v.y);
        *p = o;
    }
};
template <>
struct io<b2> {
    __device__ __forceinline__ static float2 ld(const b2* p) {
        b2 v = *p;
        return make_float2(bf16_to_f(v.x), bf16_to_f(v.y));
    }
    __device__ __forceinline__ static void st(b2* p, float2 v) {
        b2 o;
        o.x = f_to_bf16(v.x);
        o.y = f_to_bf16(v.y);
        *p = o;
    }
};

inline size_t storage_bytes(int prec) {
    switch (prec) {
        case LQT_F64: return 16;
        case LQT_F32: return 8;
        default: return 4;
    }
}

// ------------------------------------------------------------------ geometry
constexpr int LQT_MAXLAT = 8;  // lattices of one context

// Every lattice of a context, as the kernels see it (passed by value).  Lattice k owns the
// device sites [off[k], off[k] + L0 L1 L2 L3); off[k] is a multiple of 256 so that no site
// block straddles two lattices, and the sites between lattices are padding (zero fields).
struct LatTab {
    int nlat;
    int L[LQT_MAXLAT][4];
    int off[LQT_MAXLAT + 1];  // off[nlat] = V, the padded total
    int coff[LQT_MAXLAT + 1]; // first site of lattice k in the canonical layout (no padding)
    double diag[LQT_MAXLAT];  // 4 + m_k
};

struct Geom {
    int L[4];  // lattice 0 (the only one of a single-lattice context)
    int V;     // device sites of all lattices with padding
    LatTab lat;
    long long canon_sites;  // sites of all lattices without padding (canonical layout)
};

// lattice of device site s (every lattice of a context, at most LQT_MAXLAT)
__device__ __forceinline__ int lat_of(const LatTab& t, uint32_t s) {
    int k = 0;
#pragma unroll
    for (int i = 1; i < LQT_MAXLAT; i++)
        if (i < t.nlat && s >= (uint32_t)t.off[i]) k = i;
    return k;
}
// site of s within its lattice k; false for a padding site
__device__ __forceinline__ bool lat_site(const LatTab& t, uint32_t s, int& k, uint32_t& sl) {
    k = lat_of(t, s);
    sl = s - (uint32_t)t.off[k];
    return sl < (uint32_t)(t.L[k][0] * t.L[k][1] * t.L[k][2] * t.L[k][3]);
}

// XCD-aware block order: hardware hands consecutive workgroup ids to the 8 XCDs in turn;
// remapping gives each XCD one contiguous range of logical blocks so neighbouring sites
// (and the links they share) stay in one L2.
__device__ __forceinline__ int xcd_block(int nlogical) {
    int b = blockIdx.x;
    int per = (nlogical + 7) >> 3;
    int l = (b & 7) * per + (b >> 3);
    return l < nlogical ? l : -1;
}
inline int xcd_grid(int nlogical) { return ((nlogical + 7) >> 3) << 3; }

// ------------------------------------------------------------------ error handling
struct Error {
    int code;
    std::string msg;
};

#define LQT_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::lqt::Error{LQT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define LQT_CHECK(cond, code, msg)                           \
    do {                                                     \
        if (!(cond)) throw ::lqt::Error{(code), (msg)};      \
    } while (0)

// Device buffer that frees itself.
struct DBuf {
    void* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void ensure(size_t bytes) {
        if (bytes <= n) return;
        reset();
        if (bytes == 0) return;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{LQT_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
        }
        n = bytes;
    }
    template <typename T>
    T* as() const {
        return (T*)p;
    }
};

// Pinned host buffer.
struct HBuf {
    void* p = nullptr;
    size_t n = 0;
    HBuf() = default;
    HBuf(const HBuf&) = delete;
    HBuf& operator=(const HBuf&) = delete;
    ~HBuf() {
        if (p) (void)hipHostFree(p);
    }
    void ensure(size_t bytes) {
        if (bytes <= n) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess)
            throw Error{LQT_ENOMEM, "hipHostMalloc failed"};
        n = bytes;
    }
    template <typename T>
    T* as() const {
        return (T*)p;
    }
};

// Kernel families timed by KTimer.
enum {
    KT_DSLASH = 0,  // Wilson operator of the inner cycles (any storage precision)
    KT_DOTS = 1,    // CGS dot pass
    KT_UPDATE = 2,  // CGS update pass
    KT_RESID = 3,   // FP64 residual b - A x with norms (defect correction)
    KT_KRYLOV = 4,  // other Krylov kernels (cycle start, solution update, small reductions)
    KT_PROJ = 5,    // deflation projections (FP64 MFMA)
    KT_PR = 6,      // prolongator restrict / prolong
    KT_NET = 7,     // transport-network preconditioner
    KT_GRAPH = 8,   // graph-captured inner cycles (every kernel of a cycle in one launch)
    KT_N = 9
};

// Non-blocking kernel timer: event pairs recorded around launches on the context stream,
// folded into per-family totals (time, launches, algorithmic bytes) only when the pool
// fills or the totals are read.
struct KTimer {
    static constexpr int POOL = 4096;
    bool on = false;
    std::vector<hipEvent_t> e0, e1;
    std::vector<int> fam;
    std::vector<double> byt;
    int used = 0;
    int open_fam = -1;
    double ms[KT_N] = {};
    long long calls[KT_N] = {};
    double bytes[KT_N] = {};
    void init() {
        if (!e0.empty()) return;
        e0.resize(POOL);
        e1.resize(POOL);
        fam.resize(POOL);
        byt.resize(POOL);
        for (int i = 0; i < POOL; i++) {
            (void)hipEventCreate(&e0[i]);
            (void)hipEventCreate(&e1[i]);
        }
    }
    void destroy() {
        for (size_t i = 0; i < e0.size(); i++) {
            (void)hipEventDestroy(e0[i]);
            (void)hipEventDestroy(e1[i]);
        }
        e0.clear();
        e1.clear();
    }
    void flush() {
        if (used == 0) return;
        (void)hipEventSynchronize(e1[used - 1]);
        for (int i = 0; i < used; i++) {
            float t = 0;
            if (hipEventElapsedTime(&t, e0[i], e1[i]) == hipSuccess) {
                ms[fam[i]] += t;
                calls[fam[i]] += 1;
                bytes[fam[i]] += byt[i];
            }
        }
        used = 0;
    }
    void begin(hipStream_t s, int f) {
        if (!on) return;
        if (used == POOL) flush();
        (void)hipEventRecord(e0[used], s);
        fam[used] = f;
        open_fam = f;
    }
    // bytes: algorithmic HBM bytes of the launches between begin and end
    void end(hipStream_t s, double bytes_moved = 0) {
        if (!on || open_fam < 0) return;
        (void)hipEventRecord(e1[used], s);
        byt[used] = bytes_moved;
        used++;
        open_fam = -1;
    }
    void reset() {
        flush();
        for (int i = 0; i < KT_N; i++) ms[i] = 0, calls[i] = 0, bytes[i] = 0;
    }
};

struct Tuned {
    int rhs_per_thread;
    int block;
    int chunk;     // site blocks per sweep (0: site-block-major order)
    int kind = 0;  // 0 vector-ALU kernel, 1 matrix-core kernel (16-bit storage)
};

struct Net {
    bool set = false;
    std::vector<float> w;  // FP32 master weights (complex pairs), host copy
    DBuf wf;               // the weights the kernels use (BF16-rounded values held as FP32)
    DBuf act;              // two FP32 activation fields for the hidden layers
    DBuf wa;               // one layer's weights as matrix-product operands
    DBuf train[8];         // training workspace (weights, activations, deltas, Gram blocks)
};

}  // namespace lqt

struct lqt_ctx {
    lqt::Geom g;
    long long N;  // 12 V
    double mass;
    int antiperiodic;
    hipStream_t stream;
    int device;
    std::string err;
    bool have_gauge = false;
    lqt::DBuf U[4];  // gauge per precision (LQT_F64 .. LQT_BF16)
    // work buffers, grown on demand: 0 Krylov basis, 1 residuals, 2 Krylov state,
    // 3-4 Krylov partial sums, 5-6 apply / BLAS partials, 7 residual partials,
    // 8 GEMM partials, 9 small matrices, 10-11 estimator fields, 12 FGMRES preconditioned basis,
    // 13 s-step Gram partials
    lqt::DBuf scratch[14];
    lqt::HBuf pinned;
    std::map<long long, lqt::Tuned> tuned;
    lqt::KTimer timer;
    hipStream_t capture_stream = nullptr;  // private stream for graph capture (created on demand)
    lqt::Net net;
    double sigma_max = 0;  // power-iteration estimate, filled on demand
    void* blas = nullptr;  // rocBLAS handle of the dense setup eigenproblems (created on demand)
    lqt_basis* tg = nullptr;  // prolongator of the two-grid preconditioner (caller-owned)
    lqt::DBuf tg_work[2];     // its FP64 fine and coarse work fields
};

struct lqt_basis {
    lqt_ctx* ctx;
    int k = 0;
    int kind = 0;               // 0: fine vectors, 1: prolongator
    lqt::DBuf U;                // k fine vectors, device layout FP64 [k][12][V]
    std::vector<double> lambda; // 2k (complex) eigenvalues of U^+ g5 A U, ascending |.|
    std::vector<double> ug5u;   // 2k: u_i^+ g5 u_i
    bool orthonormal = false;   // Q holds an orthonormal basis (Algorithm 1 projector)
    lqt::DBuf Q;                // k orthonormal Ritz vectors of A g5 (eigensolver bases)
    std::vector<double> theta;  // Ritz values of A g5
    std::vector<double> resid;  // ||A g5 q - theta q||
    // prolongator data
    int block[4] = {0, 0, 0, 0};
    int nv = 0;
    int nagg = 0;
    lqt::DBuf W;  // [agg][chi][nv][bsites][2][3] complex double
    lqt::DBuf Wf; // FP32 copy
    lqt::DBuf Uc; // coarse eigenvectors (k x Nc) FP64
    lqt::DBuf Dc; // explicit coarse operator W^+ A W: [agg][9 stencil slots][2nv][2nv] FP64
    double coarse_build_s = 0;  // seconds spent building Dc
    // second level (blocks of the coarse lattice): nv2 = 0 when absent
    int block2[4] = {0, 0, 0, 0};
    int nv2 = 0;
    lqt::DBuf W2;   // [A][chi][nv2][bsites2 * nv][..] complex double
    lqt::DBuf Dc2;  // level-2 operator W2^+ Dc W2 as a 9-point block stencil [A][slot][2nv2][2nv2]
    double level2_build_s = 0;
};

namespace lqt {

// ---- static workspace of lqt_gram_noalloc (noalloc.hip)
#define LQT_STATIC_SCRATCH_BYTES (32u << 20)
// look up the workspace's device address on `device` (current) once; called by lqt_create
void static_scratch_init(int device);

// ---- layout (layout.hip)
void gauge_upload(lqt_ctx* c, const double* links, int on_device, double* max_unit_err, double* max_det_err);
void to_device_layout(lqt_ctx* c, const double2* canon, double2* dev, int nrhs);
void from_device_layout(lqt_ctx* c, const double2* dev, double2* canon, int nrhs);
template <typename S>
void convert_in_c64(lqt_ctx* c, const float2* canon, S* dev, int nrhs);
template <typename S>
void convert_out_c64(lqt_ctx* c, const S* dev, float2* canon, int nrhs);

// ---- dslash (dslash.hip): out = op(in), device layout, nrhs fields
// out = scale * (op(in) - shift * in) for op = A (shift, scale apply to A only)
void dslash(lqt_ctx* c, int prec, int op, const void* in, void* out, int nrhs, long long in_stride,
            long long out_stride, double shift = 0.0, double scale = 1.0);
double dslash_tune(lqt_ctx* c, int prec, int nrhs, Tuned* chosen = nullptr);
// key of the tuned-tile map for (precision, right-hand sides)
long long tune_key(int prec, int nrhs);
// tune the FP64 residual (r = b - A x with norms) for nrhs right-hand sides
double residual_tune(lqt_ctx* c, int nrhs);
// FP64 residual r = b - A x for nrhs fields and squared norms (device layout FP64).
// act maps slot -> field index (nullptr = identity).
// act (device, may be null) maps slot -> field index of b and x; r is slot-ordered.
// r = b - A x (FP64) for the fields act[0..nrhs) of b and x (act null: 0..nrhs), written
// to r[0..nrhs); rnorm2[q] = |r_q|^2 and, if given, rnorm2_lat[q * nlat + k] over lattice k
void residual64(lqt_ctx* c, const double2* b, const double2* x, double2* r, double* rnorm2, int nrhs,
                const int* act = nullptr, double* rnorm2_lat = nullptr);

}  // namespace lqt

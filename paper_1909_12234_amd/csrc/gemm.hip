// Tall-skinny FP64 products for the deflation projections, on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64, wave64).
//
// Fields are device-layout FP64 complex vectors of length n = 12 V; the contraction index
// kk runs over comp * V + site, so every vector is contiguous in kk.
//   gram     C = X^+ Y          (ka x kb)   split over kk, partial tiles summed in order
//   probes   C_up = X^+ P_+ Z, C_dn = X^+ P_- Z, Z the Rademacher probes regenerated in
//            registers (spins {0,1} -> up, {2,3} -> dn), so X^+ Z = C_up + C_dn and
//            X^+ g5 Z = C_up - C_dn come from one pass over X (Section 2.2: the k x s
//            products are all the deflation needs after the solves)
//   combine  Y = beta Y + alpha X C  (kb outputs from ka inputs)
// A complex product is four real MFMAs: re += Xr Yr + Xi Yi, im += Xr Yi - Xi Yr.
//
// Operand layout of the 16x16x4 FP64 instruction (lane l):
//   A[i][k]: i = l % 16, k = l / 16     B[k][j]: k = l / 16, j = l % 16
//   D[i][j]: j = l % 16, i = l / 16 + 4 v for the four accumulator values v
//   (checked on the device against a host product: rows are interleaved by four).
#include "gemm.h"
#include "lqt_internal.h"

namespace lqt {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint64_t gsm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int NB = 4;          // 16-column tiles per wave
constexpr long long KC = 8192; // contraction chunk per block

// ---------------------------------------------------------------- C = X^+ Y
// chunk z of the contraction index covers [z kc, (z + 1) kc), kc a multiple of 4
__global__ __launch_bounds__(256) void k_gram_part(const double2* __restrict__ X, int ka, const double2* __restrict__ Y,
                                                   int kb, long long n, long long kc, double2* __restrict__ part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int a0 = blockIdx.x * 64 + 16 * w;
    const int b0 = blockIdx.y * 16 * NB;
    const long long kbeg = (long long)blockIdx.z * kc;
    const long long kend = min(n, kbeg + kc);
    d4 ar[NB], ai[NB];
#pragma unroll
    for (int t = 0; t < NB; t++) ar[t] = ai[t] = d4{0, 0, 0, 0};
    const int a = a0 + i;
    const double2* xrow = X + (long long)min(a, ka - 1) * n;
    for (long long k0 = kbeg; k0 < kend; k0 += 4) {
        const long long kk = k0 + kq;
        const bool ok = kk < kend;
        double2 xv = (a < ka && ok) ? xrow[kk] : make_double2(0, 0);
#pragma unroll
        for (int t = 0; t < NB; t++) {
            const int b = b0 + 16 * t + i;
            double2 yv = (b < kb && ok) ? Y[(long long)b * n + kk] : make_double2(0, 0);
            ar[t] = mfma(xv.x, yv.x, ar[t]);
            ar[t] = mfma(xv.y, yv.y, ar[t]);
            ai[t] = mfma(xv.x, yv.y, ai[t]);
            ai[t] = mfma(-xv.y, yv.x, ai[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NB; t++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = a0 + kq + 4 * v, col = b0 + 16 * t + i;
            if (row < ka && col < kb)
                part[((long long)blockIdx.z * ka + row) * kb + col] = make_double2(ar[t][v], ai[t][v]);
        }
}

// ---------------------------------------------------------------- C_up/dn = X^+ P_+/- Z
__global__ __launch_bounds__(256) void k_probe_part(const double2* __restrict__ X, int ka, uint64_t seed,
                                                    long long j0, int kb, int V, double2* __restrict__ pup,
                                                    double2* __restrict__ pdn) {
    const long long n = 12LL * V;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int a0 = blockIdx.x * 64 + 16 * w;
    const int b0 = blockIdx.y * 16 * NB;
    const long long kbeg = (long long)blockIdx.z * KC;
    const long long kend = min(n, kbeg + KC);
    d4 ur[NB], ui[NB], dr[NB], di[NB];
#pragma unroll
    for (int t = 0; t < NB; t++) ur[t] = ui[t] = dr[t] = di[t] = d4{0, 0, 0, 0};
    const int a = a0 + i;
    const double2* xrow = X + (long long)min(a, ka - 1) * n;
    for (long long k0 = kbeg; k0 < kend; k0 += 4) {
        const long long kk = k0 + kq;
        const bool ok = kk < kend;
        double2 xv = (a < ka && ok) ? xrow[kk] : make_double2(0, 0);
        const int comp = ok ? (int)(kk / V) : 0;
        const long long site = ok ? kk - (long long)comp * V : 0;
        const uint64_t hi = gsm64((uint64_t)(12 * site + comp));
        const bool up = comp < 6;
        // the step's 4 entries (one per lane quarter) lie on one side of the spin split unless
        // they straddle 6V: then only the products of that side are formed (wave-uniform)
        const long long split = 6LL * V;
        const int side = (k0 + 3 < split) ? 1 : (k0 >= split ? 2 : 0);
#pragma unroll
        for (int t = 0; t < NB; t++) {
            const int b = b0 + 16 * t + i;
            double z = 0;
            if (b < kb && ok) z = (gsm64(seed ^ gsm64((uint64_t)(j0 + b) ^ hi)) >> 63) ? -1.0 : 1.0;
            if (side == 1) {
                ur[t] = mfma(xv.x, z, ur[t]);
                ui[t] = mfma(-xv.y, z, ui[t]);
            } else if (side == 2) {
                dr[t] = mfma(xv.x, z, dr[t]);
                di[t] = mfma(-xv.y, z, di[t]);
            } else {
                const double zu = up ? z : 0.0, zd = up ? 0.0 : z;
                ur[t] = mfma(xv.x, zu, ur[t]);
                ui[t] = mfma(-xv.y, zu, ui[t]);
                dr[t] = mfma(xv.x, zd, dr[t]);
                di[t] = mfma(-xv.y, zd, di[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NB; t++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = a0 + kq + 4 * v, col = b0 + 16 * t + i;
            if (row < ka && col < kb) {
                long long o = ((long long)blockIdx.z * ka + row) * kb + col;
                pup[o] = make_double2(ur[t][v], ui[t][v]);
                pdn[o] = make_double2(dr[t][v], di[t][v]);
            }
        }
}

// out[e] = sum_c part[c][e], e < ne, in chunk order (deterministic)
__global__ void k_sum_chunks(const double2* __restrict__ part, int nchunk, long long ne, double2* __restrict__ out) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double a = 0, b = 0;
    for (int c = 0; c < nchunk; c++) {
        double2 p = part[(long long)c * ne + e];
        a += p.x;
        b += p.y;
    }
    out[e] = make_double2(a, b);
}

// ---------------------------------------------------------------- Y = beta Y + alpha X C
__global__ __launch_bounds__(256) void k_combine(const double2* __restrict__ X, int ka, const double2* __restrict__ C,
                                                 int kb, long long n, double beta, double alpha,
                                                 double2* __restrict__ Y) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const long long kk0 = (long long)blockIdx.x * 64 + 16 * w;
    const int b0 = blockIdx.y * 16 * NB;
    d4 yr[NB], yi[NB];
#pragma unroll
    for (int t = 0; t < NB; t++) yr[t] = yi[t] = d4{0, 0, 0, 0};
    const long long kk = kk0 + i;
    for (int a0 = 0; a0 < ka; a0 += 4) {
        const int a = a0 + kq;
        double2 xv = (a < ka && kk < n) ? X[(long long)a * n + kk] : make_double2(0, 0);
#pragma unroll
        for (int t = 0; t < NB; t++) {
            const int b = b0 + 16 * t + i;
            double2 cv = (a < ka && b < kb) ? C[(long long)a * kb + b] : make_double2(0, 0);
            yr[t] = mfma(xv.x, cv.x, yr[t]);
            yr[t] = mfma(-xv.y, cv.y, yr[t]);
            yi[t] = mfma(xv.x, cv.y, yi[t]);
            yi[t] = mfma(xv.y, cv.x, yi[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NB; t++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const long long k = kk0 + kq + 4 * v;
            const int b = b0 + 16 * t + i;
            if (k < n && b < kb) {
                double2* p = Y + (long long)b * n + k;
                double2 o = make_double2(alpha * yr[t][v], alpha * yi[t][v]);
                if (beta != 0.0) {
                    double2 q = *p;
                    o.x += beta * q.x;
                    o.y += beta * q.y;
                }
                *p = o;
            }
        }
}

// ---------------------------------------------------------------- host side
static int nchunks(long long n) { return (int)((n + KC - 1) / KC); }

void gemm_gram(lqt_ctx* c, const double2* X, int ka, const double2* Y, int kb, double2* C_dev, long long n) {
    if (ka <= 0 || kb <= 0) return;
    if (n < 0) n = 12LL * c->g.V;
    const int nc = nchunks(n);
    c->scratch[8].ensure(sizeof(double2) * (size_t)nc * ka * kb);
    dim3 grid((ka + 63) / 64, (kb + 16 * NB - 1) / (16 * NB), nc);
    c->timer.begin(c->stream, KT_PROJ);
    hipLaunchKernelGGL(k_gram_part, grid, dim3(256), 0, c->stream, X, ka, Y, kb, n, KC, c->scratch[8].as<double2>());
    LQT_HIP(hipGetLastError());
    long long ne = (long long)ka * kb;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream,
                       c->scratch[8].as<double2>(), nc, ne, C_dev);
    LQT_HIP(hipGetLastError());
    c->timer.end(c->stream);
}

void gemm_gram_into(hipStream_t st, const double2* X, int ka, const double2* Y, int kb, long long n, int nc,
                    double2* part, double2* C_dev) {
    const long long kc = (((n + nc - 1) / nc) + 3) / 4 * 4;
    dim3 grid((ka + 63) / 64, (kb + 16 * NB - 1) / (16 * NB), nc);
    hipLaunchKernelGGL(k_gram_part, grid, dim3(256), 0, st, X, ka, Y, kb, n, kc, part);
    LQT_HIP(hipGetLastError());
    const long long ne = (long long)ka * kb;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, part, nc, ne, C_dev);
    LQT_HIP(hipGetLastError());
}

void gemm_probes(lqt_ctx* c, const double2* X, int ka, uint64_t seed, long long j0, int s, double2* Cup_dev,
                 double2* Cdn_dev) {
    if (ka <= 0 || s <= 0) return;
    const long long n = 12LL * c->g.V;
    const int nc = nchunks(n);
    const long long ne = (long long)ka * s;
    c->scratch[8].ensure(sizeof(double2) * (size_t)nc * ne * 2);
    double2* pup = c->scratch[8].as<double2>();
    double2* pdn = pup + (size_t)nc * ne;
    dim3 grid((ka + 63) / 64, (s + 16 * NB - 1) / (16 * NB), nc);
    c->timer.begin(c->stream, KT_PROJ);
    hipLaunchKernelGGL(k_probe_part, grid, dim3(256), 0, c->stream, X, ka, seed, j0, s, c->g.V, pup, pdn);
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream, pup, nc, ne,
                       Cup_dev);
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream, pdn, nc, ne,
                       Cdn_dev);
    LQT_HIP(hipGetLastError());
    c->timer.end(c->stream);
}

void gemm_combine(lqt_ctx* c, const double2* X, int ka, const double2* C_dev, int kb, double beta, double alpha,
                  double2* Y, long long n) {
    if (kb <= 0) return;
    if (n < 0) n = 12LL * c->g.V;
    dim3 grid((unsigned)((n + 63) / 64), (kb + 16 * NB - 1) / (16 * NB));
    c->timer.begin(c->stream, KT_PROJ);
    hipLaunchKernelGGL(k_combine, grid, dim3(256), 0, c->stream, X, ka, C_dev, kb, n, beta, alpha, Y);
    LQT_HIP(hipGetLastError());
    c->timer.end(c->stream);
}

}  // namespace lqt

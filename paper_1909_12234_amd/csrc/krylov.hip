// Batched restarted GMRES building blocks (gfx950).
//
// A batch of `ns` systems ("slots") advances in lock step.  The Krylov basis of slot q is
// stored as V[i][q][comp][site] in storage type S (the dot and update passes only need
// every vector of a slot in the same layout).  Stored vectors are not unit vectors:
// the true basis vector is v_i = sc[i] * vhat_i, and every stored vector is written with
// norm ~ sqrt(N) so that 16-bit storage neither overflows nor underflows.  With w = A v_j
// computed on stored vectors (true w = sc_j * what):
//   d_i        = vhat_i^+ what                         (dot pass, FP32 per lane, FP64 sums)
//   H[i][j]    = sc_i sc_j d_i
//   what'      = what - sum_i sc_i^2 d_i vhat_i        (update pass)
//   nu^2       = |what|^2 - sum_i sc_i^2 |d_i|^2       (used only to pick a write scale)
//   vhat_{j+1} = what' sqrt(N) / nu,  mu = |vhat_{j+1}|^2 (of the rounded stored values)
//   sc_{j+1}   = 1/sqrt(mu),  H[j+1][j] = sc_j nu sqrt(mu) / sqrt(N)
// The Hessenberg matrix is reduced with complex Givens rotations on the device, one
// thread per slot, so a cycle needs no host round trip except the convergence flag.
#include "lqt_internal.h"
#include "krylov.h"
#include "sstep_small.h"

namespace lqt {

template <typename C>
struct cx {
    C x, y;
};

template <typename S, typename C>
__device__ __forceinline__ cx<C> ldk(const S* p) {
    if constexpr (sizeof(S) == 16) {
        double2 v = *(const double2*)p;
        return {(C)v.x, (C)v.y};
    } else {
        float2 v = io<S>::ld(p);
        return {(C)v.x, (C)v.y};
    }
}
template <typename S, typename C>
__device__ __forceinline__ cx<C> stk(S* p, cx<C> v) {  // store and return what was stored
    if constexpr (sizeof(S) == 16) {
        *(double2*)p = make_double2((double)v.x, (double)v.y);
        return v;
    } else {
        io<S>::st(p, make_float2((float)v.x, (float)v.y));
        float2 r = io<S>::ld(p);
        return {(C)r.x, (C)r.y};
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------- 16-byte lanes
// SP = 16 / sizeof(S) complex values per 16-byte load (4 for BF16/FP16, 2 for FP32, 1 for FP64).
template <typename S>
struct Lanes {
    static constexpr int SP = 16 / (int)sizeof(S);
};

// the 16 raw bytes, and their SP complex values (loads issued together, converted after)
template <typename S>
__device__ __forceinline__ uint4 ld16raw(const S* p) {
    return *reinterpret_cast<const uint4*>(p);
}
template <typename S, typename C, int SP>
__device__ __forceinline__ void cvt16(uint4 r, cx<C> o[SP]) {
    if constexpr (SP == 1) {
        const double2 v = __builtin_bit_cast(double2, r);
        o[0] = {(C)v.x, (C)v.y};
    } else {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
        if constexpr (sizeof(S) == 8) {  // float2 x 2
            o[0] = {(C)__uint_as_float(w[0]), (C)__uint_as_float(w[1])};
            o[1] = {(C)__uint_as_float(w[2]), (C)__uint_as_float(w[3])};
        } else if constexpr (std::is_same<S, b2>::value) {
#pragma unroll
            for (int k = 0; k < 4; k++)
                o[k] = {(C)__uint_as_float(w[k] << 16), (C)__uint_as_float(w[k] & 0xffff0000u)};
        } else {  // two FP16
#pragma unroll
            for (int k = 0; k < 4; k++) {
                __half_raw lo, hi;
                lo.x = (unsigned short)(w[k] & 0xffffu);
                hi.x = (unsigned short)(w[k] >> 16);
                o[k] = {(C)__half2float(__half(lo)), (C)__half2float(__half(hi))};
            }
        }
    }
}
template <typename S, typename C, int SP>
__device__ __forceinline__ void ld16(const S* p, cx<C> o[SP]) {
    cvt16<S, C, SP>(ld16raw(p), o);
}

// store SP values, return (through o) what the storage type holds after rounding
template <typename S, typename C, int SP>
__device__ __forceinline__ void st16(S* p, cx<C> o[SP]) {
    if constexpr (SP == 1) {
        o[0] = stk<S, C>(p, o[0]);
    } else {
        uint32_t w[4];
        if constexpr (sizeof(S) == 8) {
            w[0] = __float_as_uint((float)o[0].x), w[1] = __float_as_uint((float)o[0].y);
            w[2] = __float_as_uint((float)o[1].x), w[3] = __float_as_uint((float)o[1].y);
        } else if constexpr (std::is_same<S, b2>::value) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint16_t a = f_to_bf16((float)o[k].x), b = f_to_bf16((float)o[k].y);
                w[k] = (uint32_t)a | ((uint32_t)b << 16);
                o[k] = {(C)bf16_to_f(a), (C)bf16_to_f(b)};
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                __half_raw a = __half(__float2half_rn((float)o[k].x)), b = __half(__float2half_rn((float)o[k].y));
                w[k] = (uint32_t)a.x | ((uint32_t)b.x << 16);
                o[k] = {(C)__half2float(__half(a)), (C)__half2float(__half(b))};
            }
        }
        *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// ---------------------------------------------------------------------------- flat passes
// The dot and update passes see a slot vector as n * sizeof(S) / 16 chunks of 16 bytes (SP
// complex values each; 12 V sizeof(S) is always a multiple of 16).  A block covers KTILE
// consecutive chunks of every vector, KCH per thread (strided by 256 so that each load
// instruction of a wave reads 1 KiB contiguously), and keeps its chunks of w in registers
// across the loop over the basis.  Lane partial sums are reduced across the wave with DPP
// (no LDS traffic per basis vector).
constexpr int KCH = 4;
constexpr int KTILE = 256 * KCH;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
// sum over the 64 lanes (every lane active), returned in every lane
__device__ __forceinline__ float wave_sum_f(float v) {
    v += dpp_f<0xB1>(v);         // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);         // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);        // row_half_mirror: sums of 8
    v += dpp_f<0x140>(v);        // row_mirror: sums of 16 (every lane of a row)
    v += dpp_f<0x142, 0xA>(v);   // row_bcast15 into rows 1, 3
    v += dpp_f<0x143, 0xC>(v);   // row_bcast31 into rows 2, 3: lane 63 holds the total
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <typename C>
__device__ __forceinline__ double wsum(C v) {
    if constexpr (sizeof(C) == 4)
        return (double)wave_sum_f(v);
    else
        return wave_sum(v);
}

// dot pass: part[(q*nsb + blk)*(j+2) + i] = (vhat_i^+ what) over the block's chunks for
// i <= j, and (|what|^2, 0) at i = j+1
template <typename S>
__global__ __launch_bounds__(256) void k_cgs_dots(const S* __restrict__ Vb, long long vstride, int j, long long nch,
                                                  double2* __restrict__ part) {
    using C = typename acc_of<S>::type;
    constexpr int SP = Lanes<S>::SP;
    __shared__ double red[4][KRY_MAXM + 2][2];
    const int q = blockIdx.y;
    const int nsb = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long n = nch * SP;
    const long long k0 = (long long)blockIdx.x * KTILE + threadIdx.x;
    const S* w = Vb + (long long)(j + 1) * vstride + q * n;
    cx<C> wv[KCH][SP];
    double nw = 0;
#pragma unroll
    for (int c = 0; c < KCH; c++) {
        const long long k = k0 + 256 * c;
        if (k < nch)
            ld16<S, C, SP>(w + k * SP, wv[c]);
        else
#pragma unroll
            for (int t = 0; t < SP; t++) wv[c][t] = {0, 0};
#pragma unroll
        for (int t = 0; t < SP; t++) nw += (double)wv[c][t].x * wv[c][t].x + (double)wv[c][t].y * wv[c][t].y;
    }
    int i = 0;
    for (; i + 1 <= j; i += 2) {  // two basis vectors per trip: twice the loads in flight
        const S* v0 = Vb + (long long)i * vstride + q * n;
        const S* v1 = v0 + vstride;
        C r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            const long long k = k0 + 256 * c;
            if (k < nch) {
                cx<C> a[SP], b[SP];
                ld16<S, C, SP>(v0 + k * SP, a);
                ld16<S, C, SP>(v1 + k * SP, b);
#pragma unroll
                for (int t = 0; t < SP; t++) {
                    r0 += a[t].x * wv[c][t].x + a[t].y * wv[c][t].y;
                    i0 += a[t].x * wv[c][t].y - a[t].y * wv[c][t].x;
                    r1 += b[t].x * wv[c][t].x + b[t].y * wv[c][t].y;
                    i1 += b[t].x * wv[c][t].y - b[t].y * wv[c][t].x;
                }
            }
        }
        const double s0 = wsum(r0), s1 = wsum(i0), s2 = wsum(r1), s3 = wsum(i1);
        if (lane == 0) {
            red[wave][i][0] = s0;
            red[wave][i][1] = s1;
            red[wave][i + 1][0] = s2;
            red[wave][i + 1][1] = s3;
        }
    }
    if (i <= j) {
        const S* v0 = Vb + (long long)i * vstride + q * n;
        C r0 = 0, i0 = 0;
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            const long long k = k0 + 256 * c;
            if (k < nch) {
                cx<C> a[SP];
                ld16<S, C, SP>(v0 + k * SP, a);
#pragma unroll
                for (int t = 0; t < SP; t++) {
                    r0 += a[t].x * wv[c][t].x + a[t].y * wv[c][t].y;
                    i0 += a[t].x * wv[c][t].y - a[t].y * wv[c][t].x;
                }
            }
        }
        const double s0 = wsum(r0), s1 = wsum(i0);
        if (lane == 0) {
            red[wave][i][0] = s0;
            red[wave][i][1] = s1;
        }
    }
    nw = wave_sum(nw);
    if (lane == 0) {
        red[wave][j + 1][0] = nw;
        red[wave][j + 1][1] = 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j + 1; t += 256) {
        const double a = red[0][t][0] + red[1][t][0] + red[2][t][0] + red[3][t][0];
        const double b = red[0][t][1] + red[1][t][1] + red[2][t][1] + red[3][t][1];
        part[((long long)q * nsb + blockIdx.x) * (j + 2) + t] = make_double2(a, b);
    }
}

// One block (256 threads) per slot: finish the sums, fill column j of H, the update
// coefficients alpha_i = sc_i^2 d_i and the write scale fac = sqrt(N)/nu.
// pass 0 overwrites H[:, j], pass 1 (re-orthogonalisation) adds to it.
__global__ __launch_bounds__(256) void k_cgs_finish(const double2* __restrict__ part, int nsb, int j, KryState st,
                                                    int pass, double sqrtN) {
    const int q = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ double2 d[KRY_MAXM + 2];
    for (int i = wave; i <= j + 1; i += 4) {  // one wave per basis index
        double a = 0, b = 0;
        for (int k = lane; k < nsb; k += 64) {
            double2 p = part[((long long)q * nsb + k) * (j + 2) + i];
            a += p.x;
            b += p.y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) d[i] = make_double2(a, b);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int m = st.m;
    double* sc = st.sc + (long long)q * (m + 1);
    double2* H = st.H + (long long)q * (m + 1) * m;
    double2* alpha = st.alpha + (long long)q * (m + 1);
    if (st.frozen[q]) {  // cycle of this slot has ended: keep its (unused) vectors finite
        for (int i = 0; i <= j; i++) alpha[i] = make_double2(0, 0);
        st.fac[q] = 1.0;
        st.nu[q] = 1.0;
        return;
    }
    double nu2 = d[j + 1].x;
    for (int i = 0; i <= j; i++) {
        double f = sc[i] * sc[j];
        double2 h = make_double2(f * d[i].x, f * d[i].y);
        if (pass == 0)
            H[i * m + j] = h;
        else
            H[i * m + j] = make_double2(H[i * m + j].x + h.x, H[i * m + j].y + h.y);
        double g = sc[i] * sc[i];
        alpha[i] = make_double2(g * d[i].x, g * d[i].y);
        nu2 -= g * (d[i].x * d[i].x + d[i].y * d[i].y);
    }
    double floor2 = 1e-10 * d[j + 1].x;
    if (!(nu2 > floor2)) nu2 = floor2 > 0 ? floor2 : 1e-300;
    st.fac[q] = sqrtN / sqrt(nu2);
    st.nu[q] = sqrt(nu2);
}

// update pass: what' = what - sum_i alpha_i vhat_i, optionally scaled by fac and stored;
// part[q*nsb + blk] = |stored|^2 over the block's chunks (of the rounded stored values)
template <typename S>
__global__ __launch_bounds__(256) void k_cgs_update(S* __restrict__ Vb, long long vstride, int j, long long nch,
                                                    KryState st, int scale, double* __restrict__ part) {
    using C = typename acc_of<S>::type;
    constexpr int SP = Lanes<S>::SP;
    __shared__ double red[4];
    const int q = blockIdx.y;
    const int nsb = gridDim.x;
    const int m = st.m;
    const long long n = nch * SP;
    const long long k0 = (long long)blockIdx.x * KTILE + threadIdx.x;
    S* w = Vb + (long long)(j + 1) * vstride + q * n;
    const double2* alpha = st.alpha + (long long)q * (m + 1);
    cx<C> wv[KCH][SP];
#pragma unroll
    for (int c = 0; c < KCH; c++) {
        const long long k = k0 + 256 * c;
        if (k < nch)
            ld16<S, C, SP>(w + k * SP, wv[c]);
        else
#pragma unroll
            for (int t = 0; t < SP; t++) wv[c][t] = {0, 0};
    }
    int i = 0;
    for (; i + 1 <= j; i += 2) {
        const double2 a0 = alpha[i], a1 = alpha[i + 1];
        const C ar = (C)a0.x, ai = (C)a0.y, br = (C)a1.x, bi = (C)a1.y;
        const S* v0 = Vb + (long long)i * vstride + q * n;
        const S* v1 = v0 + vstride;
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            const long long k = k0 + 256 * c;
            if (k < nch) {
                cx<C> a[SP], b[SP];
                ld16<S, C, SP>(v0 + k * SP, a);
                ld16<S, C, SP>(v1 + k * SP, b);
#pragma unroll
                for (int t = 0; t < SP; t++) {
                    wv[c][t].x -= ar * a[t].x - ai * a[t].y + br * b[t].x - bi * b[t].y;
                    wv[c][t].y -= ar * a[t].y + ai * a[t].x + br * b[t].y + bi * b[t].x;
                }
            }
        }
    }
    if (i <= j) {
        const double2 a0 = alpha[i];
        const C ar = (C)a0.x, ai = (C)a0.y;
        const S* v0 = Vb + (long long)i * vstride + q * n;
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            const long long k = k0 + 256 * c;
            if (k < nch) {
                cx<C> a[SP];
                ld16<S, C, SP>(v0 + k * SP, a);
#pragma unroll
                for (int t = 0; t < SP; t++) {
                    wv[c][t].x -= ar * a[t].x - ai * a[t].y;
                    wv[c][t].y -= ar * a[t].y + ai * a[t].x;
                }
            }
        }
    }
    const C f = scale ? (C)st.fac[q] : (C)1;
    double nrm = 0;
#pragma unroll
    for (int c = 0; c < KCH; c++) {
        const long long k = k0 + 256 * c;
        if (k < nch) {
#pragma unroll
            for (int t = 0; t < SP; t++) wv[c][t] = {wv[c][t].x * f, wv[c][t].y * f};
            st16<S, C, SP>(w + k * SP, wv[c]);
#pragma unroll
            for (int t = 0; t < SP; t++) nrm += (double)wv[c][t].x * wv[c][t].x + (double)wv[c][t].y * wv[c][t].y;
        }
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)q * nsb + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}


// One block (64 threads) per slot: mu, sc_{j+1}, H[j+1][j], then the Givens step.
__global__ void k_norm_givens(const double* __restrict__ part, int nsb, int j, KryState st, double sqrtN) {
    const int q = blockIdx.x;
    double a = 0;
    for (int k = threadIdx.x; k < nsb; k += 64) a += part[(long long)q * nsb + k];
    a = wave_sum(a);
    if (threadIdx.x != 0) return;
    const int m = st.m;
    double* sc = st.sc + (long long)q * (m + 1);
    double2* H = st.H + (long long)q * (m + 1) * m;
    double* cs = st.cs + (long long)q * m;
    double2* sn = st.sn + (long long)q * m;
    double2* g = st.g + (long long)q * (m + 1);
    if (st.frozen[q]) return;  // this slot's cycle already ended
    double mu = a;
    double hn = sc[j] * st.nu[q] * sqrt(mu) / sqrtN;
    sc[j + 1] = mu > 0 ? 1.0 / sqrt(mu) : 0.0;
    H[(j + 1) * m + j] = make_double2(hn, 0);
    // previous rotations on column j: [c s; -conj(s) c]
    for (int i = 0; i < j; i++) {
        double2 h0 = H[i * m + j], h1 = H[(i + 1) * m + j];
        double c = cs[i];
        double2 s = sn[i];
        double2 t0 = make_double2(c * h0.x + s.x * h1.x - s.y * h1.y, c * h0.y + s.x * h1.y + s.y * h1.x);
        double2 t1 = make_double2(-(s.x * h0.x + s.y * h0.y) + c * h1.x, -(s.x * h0.y - s.y * h0.x) + c * h1.y);
        H[i * m + j] = t0;
        H[(i + 1) * m + j] = t1;
    }
    double2 av = H[j * m + j];
    double absa = sqrt(av.x * av.x + av.y * av.y);
    double r = sqrt(absa * absa + hn * hn);
    double c;
    double2 s;
    if (r == 0) {
        c = 1;
        s = make_double2(0, 0);
    } else if (absa == 0) {
        c = 0;
        s = make_double2(1, 0);
    } else {
        c = absa / r;
        s = make_double2(av.x / absa * hn / r, av.y / absa * hn / r);
    }
    cs[j] = c;
    sn[j] = s;
    H[j * m + j] = make_double2(c * av.x + s.x * hn, c * av.y + s.y * hn);
    H[(j + 1) * m + j] = make_double2(0, 0);
    double2 g0 = g[j];
    g[j] = make_double2(c * g0.x, c * g0.y);
    g[j + 1] = make_double2(-(s.x * g0.x + s.y * g0.y), -(s.x * g0.y - s.y * g0.x));
    double est = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
    st.est[q] = est;
    st.kdim[q] = j + 1;
    bool breakdown = !(hn > 1e-300) || !(mu > 0);
    if (est <= st.target[q] || breakdown || !(est == est)) st.frozen[q] = 1;
}

// ---------------------------------------------------------------------------- cycle ends
// Back substitution R y = g and beta_i = y_i sc_i (one thread per slot).
__global__ void k_backsolve(KryState st, int ns) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    const int m = st.m;
    const int k = st.kdim[q];
    const double2* H = st.H + (long long)q * (m + 1) * m;
    const double2* g = st.g + (long long)q * (m + 1);
    const double* sc = st.sc + (long long)q * (m + 1);
    double2* y = st.y + (long long)q * (m + 1);
    for (int i = k - 1; i >= 0; i--) {
        double2 t = g[i];
        for (int l = i + 1; l < k; l++) {
            double2 h = H[i * m + l], yl = y[l];
            t.x -= h.x * yl.x - h.y * yl.y;
            t.y -= h.x * yl.y + h.y * yl.x;
        }
        double2 d = H[i * m + i];
        double den = d.x * d.x + d.y * d.y;
        double2 v = den > 0 ? make_double2((t.x * d.x + t.y * d.y) / den, (t.y * d.x - t.x * d.y) / den)
                            : make_double2(0, 0);
        y[i] = v;
    }
    for (int i = 0; i < k; i++) st.beta[(long long)q * (m + 1) + i] = make_double2(y[i].x * sc[i], y[i].y * sc[i]);
    for (int i = k; i <= m; i++) st.beta[(long long)q * (m + 1) + i] = make_double2(0, 0);
}

// x[act[q]] += sum_i beta_i Zhat_i  (FP64 solution, basis in S; Z = V without preconditioner)
template <typename S>
__global__ __launch_bounds__(256) void k_xupdate(double2* __restrict__ x, const int* __restrict__ act,
                                                 const S* __restrict__ Zb, long long zstride, int V, KryState st) {
    const int q = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const long long n = 12LL * V;
    const int m = st.m;
    const int k = st.kdim[q];
    double2* xq = x + (long long)act[q] * n;
    double2 acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = xq[(long long)c * V + s];
    for (int i = 0; i < k; i++) {
        double2 b = st.beta[(long long)q * (m + 1) + i];
        const S* zi = Zb + (long long)i * zstride + q * n;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            cx<double> v = ldk<S, double>(zi + (long long)c * V + s);
            acc[c].x += b.x * v.x - b.y * v.y;
            acc[c].y += b.x * v.y + b.y * v.x;
        }
    }
#pragma unroll
    for (int c = 0; c < 12; c++) xq[(long long)c * V + s] = acc[c];
}

// U basis vectors of one carry trip: their loads are issued together, then
// ax += sum_u bx[i+u] k_{i+u} and ak += sum_u wk[i+u] k_{i+u} in FP64, in the order of u
template <typename S, int U, int SP>
__device__ __forceinline__ void carry_trip(const S* kq, long long kstride, int i, const double2* bx,
                                           const double2* wk, cx<double> ax[SP], cx<double> ak[SP]) {
    uint4 r[U];
#pragma unroll
    for (int u = 0; u < U; u++) r[u] = ld16raw(kq + (long long)(i + u) * kstride);
#pragma unroll
    for (int u = 0; u < U; u++) {
        cx<double> v[SP];
        cvt16<S, double, SP>(r[u], v);
        const double2 b = bx[i + u], w = wk[i + u];
#pragma unroll
        for (int t = 0; t < SP; t++) {
            ax[t].x += b.x * v[t].x - b.y * v[t].y;
            ax[t].y += b.x * v[t].y + b.y * v[t].x;
            ak[t].x += w.x * v[t].x - w.y * v[t].y;
            ak[t].y += w.x * v[t].y + w.y * v[t].x;
        }
    }
}

// End of an s-step cycle that carries the residual in the basis (reliable updates): with
// beta the cycle's coefficients (x += K_s beta) and A k_i = k_{i+1}/sigma + theta k_i for the
// stored vectors, the new residual is r - A K_s beta = rho k_0 - K_{s+1} gamma, gamma = T beta
// (gamma_i = theta beta_i + beta_{i-1}/sigma), rho = |r|/sqrt(N) of the cycle's start.  It is
// written over k_0 scaled by sqrt(N)/est (est: the cycle's least-squares residual norm, which
// the next cycle takes as its |r|), so x and the next start vector come from one pass over
// the basis.  The pass is flat over the slot's 16-byte chunks of k_i (SP complex values, one
// chunk per thread; x is read and written as the chunk's SP FP64 values) and keeps eight basis
// vectors' loads in flight per trip.  part[q * gridDim.x + blk] = partial |r_new|^2 of the
// block's 256 chunks.
template <typename S>
__global__ __launch_bounds__(256) void k_sstep_carry(double2* __restrict__ x, const int* __restrict__ act,
                                                     S* __restrict__ Kb, long long kstride, long long nch,
                                                     KryState st, double theta, double sigma, double sqrtN,
                                                     double* __restrict__ part) {
    constexpr int SP = Lanes<S>::SP;
    __shared__ double2 bx[KRY_MAXM + 1], wk[KRY_MAXM + 1];
    __shared__ double red[4];
    const int q = blockIdx.y;
    const int m = st.m;
    const int kd = st.kdim[q];
    if (threadIdx.x <= kd) {
        const int i = threadIdx.x;
        const double2* beta = st.beta + (long long)q * (m + 1);
        const double2 bi = i < kd ? beta[i] : make_double2(0, 0);
        const double2 bm = i >= 1 ? beta[i - 1] : make_double2(0, 0);
        const double est = st.est[q];
        const double f = est > 0 ? sqrtN / est : 0.0;
        const double rho = i == 0 ? st.g[(long long)q * (m + 1)].x / sqrtN : 0.0;
        bx[i] = bi;
        wk[i] = make_double2((rho - theta * bi.x - bm.x / sigma) * f, (-theta * bi.y - bm.y / sigma) * f);
    }
    __syncthreads();
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long n = nch * SP;
    double nrm = 0;
    if (k < nch) {
        double2* xq = x + (long long)act[q] * n + k * SP;
        const S* kq = Kb + q * n + k * SP;
        cx<double> ax[SP], ak[SP];
#pragma unroll
        for (int t = 0; t < SP; t++) {
            const double2 v = xq[t];
            ax[t] = {v.x, v.y};
            ak[t] = {0, 0};
        }
        int i = 0;
        for (; i + 7 <= kd; i += 8) carry_trip<S, 8, SP>(kq, kstride, i, bx, wk, ax, ak);
        if (i + 3 <= kd) {
            carry_trip<S, 4, SP>(kq, kstride, i, bx, wk, ax, ak);
            i += 4;
        }
        for (; i <= kd; i++) carry_trip<S, 1, SP>(kq, kstride, i, bx, wk, ax, ak);
#pragma unroll
        for (int t = 0; t < SP; t++) {
            xq[t] = make_double2(ax[t].x, ax[t].y);
            nrm += ak[t].x * ak[t].x + ak[t].y * ak[t].y;
        }
        st16<S, double, SP>(Kb + q * n + k * SP, ak);
    }
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sc = st.est[q] / sqrtN;
        part[(long long)q * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + (red[2] + red[3])) * sc * sc;
    }
}

// rn2[q] = sum of the nblk partials of slot q (fixed order)
__global__ void k_carry_norms(const double* __restrict__ part, int nblk, double* __restrict__ rn2) {
    __shared__ double red[256];
    const int q = blockIdx.x;
    double v = 0;
    for (int i = threadIdx.x; i < nblk; i += 256) v += part[(long long)q * nblk + i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rn2[q] = red[0];
}

// Cycle state of a slot that starts from the carried residual: k_0 already holds r sqrt(N)/est
// (est of the previous cycle), so |r| is taken as est.
__global__ void k_start_state_carry(KryState st, const double* __restrict__ target_abs, int ns, double sqrtN) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    const int m = st.m;
    const double nr = st.est[q];
    st.sc[(long long)q * (m + 1)] = 1.0 / sqrtN;
    st.g[(long long)q * (m + 1)] = make_double2(nr, 0);
    for (int i = 1; i <= m; i++) st.g[(long long)q * (m + 1) + i] = make_double2(0, 0);
    st.kdim[q] = 0;
    st.frozen[q] = nr > 0 ? 0 : 1;
    st.target[q] = target_abs[q];
}

// vhat_0[q] = r[src[q]] * sqrt(N)/|r|, in storage S.  Also resets the slot's cycle state.
template <typename S>
__global__ __launch_bounds__(256) void k_start(S* __restrict__ V0, const double2* __restrict__ r,
                                               const int* __restrict__ src, const double* __restrict__ rn2, int V,
                                               double sqrtN) {
    const int q = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const long long n = 12LL * V;
    const int sq = src[q];
    double nr = sqrt(rn2[sq]);
    double f = nr > 0 ? sqrtN / nr : 0.0;
    const double2* rq = r + (long long)sq * n;
    S* vq = V0 + (long long)q * n;
#pragma unroll
    for (int c = 0; c < 12; c++) {
        double2 v = rq[(long long)c * V + s];
        stk<S, double>(vq + (long long)c * V + s, cx<double>{v.x * f, v.y * f});
    }
}

__global__ void k_start_state(KryState st, const int* __restrict__ src, const double* __restrict__ rn2,
                              const double* __restrict__ target_abs, int ns, double sqrtN) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    const int m = st.m;
    double nr = sqrt(rn2[src[q]]);
    st.sc[(long long)q * (m + 1)] = 1.0 / sqrtN;
    st.g[(long long)q * (m + 1)] = make_double2(nr, 0);
    for (int i = 1; i <= m; i++) st.g[(long long)q * (m + 1) + i] = make_double2(0, 0);
    st.kdim[q] = 0;
    st.est[q] = nr;
    st.frozen[q] = nr > 0 ? 0 : 1;
    st.target[q] = target_abs[q];
}

// ---------------------------------------------------------------------------- s-step cycles
// The cycle's basis is k_0 = r sqrt(N)/|r|, k_{i+1} = sigma (A - theta) k_i (no Gram-Schmidt
// between the operator applications), so A k_i = k_{i+1}/sigma + theta k_i.  One pass forms
// the Gram matrix G = K^+ K; with G = R^+ R (Cholesky, FP64) K = Q R, A Q_s = Q H with
// H = R T R_s^{-1}, T[i][i] = theta, T[i+1][i] = 1/sigma, and GMRES minimises
// |rho R_00 e_1 - H y| (rho = |r|/sqrt(N)); the update is x += K_s R_s^{-1} y.

// Gram partial sums of the NV = s+1 stored vectors of slot q over the elements of block
// blk: part[(q*nblk + blk)*2*NP + 2p (+1)] for the upper-triangle pair p = (i <= j).
template <typename S, int NV>
__global__ __launch_bounds__(256) void k_sgram(const S* __restrict__ Vb, long long vstride, long long n,
                                               double* __restrict__ part) {
    using C = typename acc_of<S>::type;
    constexpr int NP = NV * (NV + 1) / 2;
    __shared__ double red[4][2 * NP];
    const int q = blockIdx.y, nblk = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long per = ((n + nblk - 1) / nblk + 255) / 256 * 256;
    const long long e0 = (long long)blockIdx.x * per, e1 = min(n, e0 + per);
    C ar[NP], ai[NP];
#pragma unroll
    for (int p = 0; p < NP; p++) ar[p] = ai[p] = 0;
    const S* base = Vb + q * n;
    for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
        cx<C> v[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) v[i] = ldk<S, C>(base + i * vstride + e);
        int p = 0;
#pragma unroll
        for (int i = 0; i < NV; i++)
#pragma unroll
            for (int j = i; j < NV; j++, p++) {
                ar[p] += v[i].x * v[j].x + v[i].y * v[j].y;
                ai[p] += v[i].x * v[j].y - v[i].y * v[j].x;
            }
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const double a = wsum(ar[p]), b = wsum(ai[p]);
        if (lane == 0) {
            red[wave][2 * p] = a;
            red[wave][2 * p + 1] = b;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 2 * NP; t += 256)
        part[((long long)q * nblk + blockIdx.x) * 2 * NP + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// Gram partials with the matrix cores, for 16-bit storage and up to 16 vectors: the rows of
// X are the real parts (rows 0..15) and the imaginary parts (rows 16..31) of k_0..k_15 (zero
// rows past s+1), X X^T accumulates in one 32x32 FP32 tile per wave over 16 elements per
// MFMA (products of 16-bit values are exact in FP32), flushed to FP64 every 1024 elements;
// G = K^+ K = (RR + II) + i (RI - IR) is written as the same upper-triangle partials as
// k_sgram.  MFMA 32x32x16 operands: lane l holds row l % 32, elements 8 (l / 32) + 0..7;
// result: lane l, register v holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
typedef __bf16 lqt_bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 lqt_h8 __attribute__((ext_vector_type(8)));

typedef float lqt_f4v __attribute__((ext_vector_type(4)));

// acc += X Y^T for two 16 x 32 tiles (row = vector, column = element): lane l holds row l % 16,
// elements 8 (l / 16) .. 8 (l / 16) + 7 of both operands
template <typename S>
__device__ __forceinline__ lqt_f4v mfma_rows(const uint32_t (&x)[4], const uint32_t (&y)[4], lqt_f4v acc) {
    if constexpr (std::is_same<S, b2>::value)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(lqt_bf8, x), __builtin_bit_cast(lqt_bf8, y),
                                                       acc, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(lqt_h8, x), __builtin_bit_cast(lqt_h8, y), acc,
                                                      0, 0, 0);
}

// Gram partial sums of up to 16 stored 16-bit vectors of slot q on the matrix cores.  A pass of
// a wave covers 32 consecutive elements of every vector: lane l loads elements 8 (l / 16) ..
// + 7 of vector l % 16 (32 bytes, each element loaded once), splits them into real and
// imaginary halves, and three 16 x 16 x 32 products accumulate RR = Re Re^T, II = Im Im^T and
// RI = Re Im^T, so G = RR + II + i (RI - RI^T).  FP32 sums are flushed to FP64 every 64
// passes; the block's four waves are summed in LDS.
template <typename S>
__global__ __launch_bounds__(256) void k_sgram_mf(const S* __restrict__ Vb, long long vstride, long long n, int nv,
                                                  double* __restrict__ part) {
    static_assert(sizeof(S) == 4, "16-bit complex storage only");
    __shared__ double red[3][16][17];
    const int q = blockIdx.y, nblk = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int vec = lane & 15, kg = lane >> 4;
    const bool live = vec < nv;
    const uint32_t* base = (const uint32_t*)(Vb + (live ? vec : 0) * vstride + q * n);
    // a wave takes GU consecutive chunks of 32 elements per pass, all loads before the products
    constexpr int GU = 4;
    const long long nch = (n + 31) / 32;
    const long long wid = (long long)blockIdx.x * 4 + wave, nw = (long long)nblk * 4;
    lqt_f4v arr = {}, aii = {}, ari = {};
    double drr[4] = {0, 0, 0, 0}, dii[4] = {0, 0, 0, 0}, dri[4] = {0, 0, 0, 0};
    int cnt = 0;
    for (long long c0 = wid * GU; c0 < nch; c0 += nw * GU) {
        uint32_t w[GU][8];
#pragma unroll
        for (int u = 0; u < GU; u++) {
            const long long e = (c0 + u) * 32 + kg * 8;
            if (live && e + 8 <= n) {
                const uint4 a = *(const uint4*)(base + e), b = *(const uint4*)(base + e + 4);
                w[u][0] = a.x, w[u][1] = a.y, w[u][2] = a.z, w[u][3] = a.w;
                w[u][4] = b.x, w[u][5] = b.y, w[u][6] = b.z, w[u][7] = b.w;
            } else {
#pragma unroll
                for (int t = 0; t < 8; t++) w[u][t] = (live && e + t < n) ? base[e + t] : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < GU; u++) {
            // 8 complex values (re low, im high 16 bits) -> packed real and imaginary halves
            uint32_t re[4], im[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                re[t] = __builtin_amdgcn_perm(w[u][2 * t + 1], w[u][2 * t], 0x05040100u);
                im[t] = __builtin_amdgcn_perm(w[u][2 * t + 1], w[u][2 * t], 0x07060302u);
            }
            arr = mfma_rows<S>(re, re, arr);
            aii = mfma_rows<S>(im, im, aii);
            ari = mfma_rows<S>(re, im, ari);
        }
        cnt += GU;
        if (cnt >= 64) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                drr[v] += arr[v], dii[v] += aii[v], dri[v] += ari[v];
                arr[v] = aii[v] = ari[v] = 0;
            }
            cnt = 0;
        }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) drr[v] += arr[v], dii[v] += aii[v], dri[v] += ari[v];
    // sum the four waves' tiles in LDS: lane l holds rows 4 (l / 16) + v, column l % 16
    for (int t = threadIdx.x; t < 3 * 16 * 17; t += 256) (&red[0][0][0])[t] = 0;
    __syncthreads();
    for (int wv = 0; wv < 4; wv++) {
        if (wave == wv)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = 4 * kg + v;
                red[0][r][vec] += drr[v];
                red[1][r][vec] += dii[v];
                red[2][r][vec] += dri[v];
            }
        __syncthreads();
    }
    const int NP = nv * (nv + 1) / 2;
    for (int p = threadIdx.x; p < NP; p += 256) {
        int i = 0, rem = p;
        while (rem >= nv - i) {
            rem -= nv - i;
            i++;
        }
        const int j = i + rem;
        double* o = part + ((long long)q * nblk + blockIdx.x) * 2 * NP;
        o[2 * p] = red[0][i][j] + red[1][i][j];
        o[2 * p + 1] = red[2][i][j] - red[2][j][i];
    }
}

template <int NV>
__global__ void k_sstep_solve(const double* __restrict__ part, int nblk, KryState st, int ns, double theta,
                              double sigma, double sqrtN) {
    constexpr int NP = NV * (NV + 1) / 2;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    const int m = st.m;
    double2 G[NV][NV];
    int p = 0;
    for (int i = 0; i < NV; i++)
        for (int j = i; j < NV; j++, p++) {
            double a = 0, b = 0;
            for (int k = 0; k < nblk; k++) {
                a += part[((long long)q * nblk + k) * 2 * NP + 2 * p];
                b += part[((long long)q * nblk + k) * 2 * NP + 2 * p + 1];
            }
            G[i][j] = make_double2(a, b);
            G[j][i] = make_double2(a, -b);
        }
    double est = 0;
    st.kdim[q] = sstep_small_solve<NV>(G, st.g[(long long)q * (m + 1)].x, theta, sigma, sqrtN, m,
                                       st.beta + (long long)q * (m + 1), &est);
    st.est[q] = est;
}

// The same small solve with one 64-thread block per system and the matrices in LDS (the
// one-thread form keeps them in private memory, which is slow for 16 x 16).
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {  // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

template <int NV>
__global__ __launch_bounds__(64) void k_sstep_solve_w(const double* __restrict__ part, int nblk, KryState st,
                                                      double theta, double sigma, double sqrtN) {
    constexpr int NP = NV * (NV + 1) / 2;
    __shared__ double2 G[NV][NV + 1], R[NV][NV + 1], Ri[NV][NV + 1], H[NV][NV + 1];
    __shared__ double2 g[NV + 1], y[NV];
    __shared__ int kk_s;
    __shared__ double cs_c;
    __shared__ double2 cs_s;
    const int q = blockIdx.x, t = threadIdx.x;
    const int m = st.m;
    // 1. Gram matrix from the block partials
    for (int p = t; p < NP; p += 64) {
        double a = 0, b = 0;
        for (int k = 0; k < nblk; k++) {
            a += part[((long long)q * nblk + k) * 2 * NP + 2 * p];
            b += part[((long long)q * nblk + k) * 2 * NP + 2 * p + 1];
        }
        int i = 0, rem = p;
        while (rem >= NV - i) {
            rem -= NV - i;
            i++;
        }
        const int j = i + rem;
        G[i][j] = make_double2(a, b);
        G[j][i] = make_double2(a, -b);
    }
    for (int e = t; e < NV * NV; e += 64) R[e / NV][e % NV] = make_double2(0, 0);
    if (t == 0) kk_s = NV;
    __syncthreads();
    // 2. Cholesky G = R^+ R, stopping at the first pivot below 1e-12 G_00
    const double floor = 1e-12 * G[0][0].x;
    for (int j = 0; j < NV; j++) {
        if (t == 0) {
            double d = G[j][j].x;
            for (int k = 0; k < j; k++) d -= R[k][j].x * R[k][j].x + R[k][j].y * R[k][j].y;
            if (!(d > floor && d < HUGE_VAL))  // tiny, negative or not finite
                kk_s = j;
            else
                R[j][j] = make_double2(sqrt(d), 0);
        }
        __syncthreads();
        if (kk_s <= j) break;
        for (int l = j + 1 + t; l < NV; l += 64) {
            double2 v = G[j][l];
            for (int k = 0; k < j; k++) {
                const double2 c = cjmul(R[k][j], R[k][l]);
                v.x -= c.x;
                v.y -= c.y;
            }
            R[j][l] = make_double2(v.x / R[j][j].x, v.y / R[j][j].x);
        }
        __syncthreads();
    }
    const int ss = kk_s - 1;
    const double nr = st.g[(long long)q * (m + 1)].x;
    double2* beta = st.beta + (long long)q * (m + 1);
    for (int i = t; i <= m; i += 64) beta[i] = make_double2(0, 0);
    if (ss < 1 || !(nr > 0)) {
        if (t == 0) {
            st.kdim[q] = 0;
            st.est[q] = nr;
        }
        return;
    }
    // 3. Ri = R_ss^{-1}, one column per thread
    for (int j = t; j < ss; j += 64) {
        for (int i = 0; i < ss; i++) Ri[i][j] = make_double2(0, 0);
        Ri[j][j] = make_double2(1.0 / R[j][j].x, 0);
        for (int i = j - 1; i >= 0; i--) {
            double2 v = make_double2(0, 0);
            for (int k = i + 1; k <= j; k++) {
                const double2 c = cmul(R[i][k], Ri[k][j]);
                v.x += c.x;
                v.y += c.y;
            }
            Ri[i][j] = make_double2(-v.x / R[i][i].x, -v.y / R[i][i].x);
        }
    }
    __syncthreads();
    // 4. H = R T Ri, (T Ri)[k][j] = theta Ri[k][j] + Ri[k-1][j] / sigma
    for (int e = t; e < (ss + 1) * ss; e += 64) {
        const int i = e / ss, j = e % ss;
        double2 h = make_double2(0, 0);
        for (int k = i; k <= ss; k++) {
            double2 tr = make_double2(0, 0);
            if (k < ss) tr = make_double2(theta * Ri[k][j].x, theta * Ri[k][j].y);
            if (k >= 1) {
                tr.x += Ri[k - 1][j].x / sigma;
                tr.y += Ri[k - 1][j].y / sigma;
            }
            const double2 c = cmul(R[i][k], tr);
            h.x += c.x;
            h.y += c.y;
        }
        H[i][j] = h;
    }
    for (int i = t; i <= ss; i += 64) g[i] = make_double2(i == 0 ? nr / sqrtN * R[0][0].x : 0.0, 0);
    __syncthreads();
    // 5. Givens QR of H against g
    for (int j = 0; j < ss; j++) {
        if (t == 0) {
            const double2 a = H[j][j], b = H[j + 1][j];
            const double absa = sqrt(a.x * a.x + a.y * a.y), absb = sqrt(b.x * b.x + b.y * b.y);
            const double r = sqrt(absa * absa + absb * absb);
            if (r == 0) {
                cs_c = 1;
                cs_s = make_double2(0, 0);
            } else if (absa == 0) {
                cs_c = 0;
                cs_s = make_double2(b.x / absb, -b.y / absb);
            } else {
                cs_c = absa / r;
                const double ux = a.x / absa, uy = a.y / absa;
                cs_s = make_double2((ux * b.x + uy * b.y) / r, (uy * b.x - ux * b.y) / r);
            }
        }
        __syncthreads();
        const double c = cs_c;
        const double2 sn = cs_s;
        for (int l = j + t; l <= ss; l += 64) {  // column l < ss of H, l == ss stands for g
            const double2 h0 = l < ss ? H[j][l] : g[j], h1 = l < ss ? H[j + 1][l] : g[j + 1];
            const double2 a0 = make_double2(c * h0.x + sn.x * h1.x - sn.y * h1.y, c * h0.y + sn.x * h1.y + sn.y * h1.x);
            const double2 a1 =
                make_double2(-(sn.x * h0.x + sn.y * h0.y) + c * h1.x, -(sn.x * h0.y - sn.y * h0.x) + c * h1.y);
            if (l < ss) {
                H[j][l] = a0;
                H[j + 1][l] = a1;
            } else {
                g[j] = a0;
                g[j + 1] = a1;
            }
        }
        __syncthreads();
    }
    // 6. back substitution, then beta = Ri y
    if (t == 0)
        for (int i = ss - 1; i >= 0; i--) {
            double2 v = g[i];
            for (int l = i + 1; l < ss; l++) {
                const double2 c = cmul(H[i][l], y[l]);
                v.x -= c.x;
                v.y -= c.y;
            }
            const double2 d = H[i][i];
            const double den = d.x * d.x + d.y * d.y;
            y[i] = den > 0 ? make_double2((v.x * d.x + v.y * d.y) / den, (v.y * d.x - v.x * d.y) / den)
                           : make_double2(0, 0);
        }
    __syncthreads();
    for (int i = t; i < ss; i += 64) {
        double2 v = make_double2(0, 0);
        for (int k = i; k < ss; k++) {
            const double2 c = cmul(Ri[i][k], y[k]);
            v.x += c.x;
            v.y += c.y;
        }
        beta[i] = v;
    }
    if (t == 0) {
        st.kdim[q] = ss;
        st.est[q] = sqrt(g[ss].x * g[ss].x + g[ss].y * g[ss].y) * sqrtN / R[0][0].x;
    }
}

// ---------------------------------------------------------------------------- host side
// chunks of 16 bytes in one slot vector (12 V complex values of S)
template <typename S>
static long long kry_chunks(const lqt_ctx* c) {
    return 12LL * c->g.V * (long long)sizeof(S) / 16;
}

// partial-sum blocks per slot of the dot and update passes
template <typename S>
int kry_blocks(const lqt_ctx* c) {
    return (int)((kry_chunks<S>(c) + KTILE - 1) / KTILE);
}

template <typename S>
void kry_dots(lqt_ctx* c, const void* Vb, long long vstride, int j, int ns, double2* part) {
    dim3 grid(kry_blocks<S>(c), ns);
    hipLaunchKernelGGL(k_cgs_dots<S>, grid, dim3(256), 0, c->stream, (const S*)Vb, vstride, j, kry_chunks<S>(c), part);
    LQT_HIP(hipGetLastError());
}
template <typename S>
void kry_update(lqt_ctx* c, void* Vb, long long vstride, int j, int ns, const KryState& st, int scale, double* part) {
    dim3 grid(kry_blocks<S>(c), ns);
    hipLaunchKernelGGL(k_cgs_update<S>, grid, dim3(256), 0, c->stream, (S*)Vb, vstride, j, kry_chunks<S>(c), st, scale,
                       part);
    LQT_HIP(hipGetLastError());
}
template <typename S>
void kry_xupdate(lqt_ctx* c, double2* x, const int* act, const void* Zb, long long zstride, int ns,
                 const KryState& st) {
    dim3 grid((c->g.V + 255) / 256, ns);
    hipLaunchKernelGGL(k_xupdate<S>, grid, dim3(256), 0, c->stream, x, act, (const S*)Zb, zstride, c->g.V, st);
    LQT_HIP(hipGetLastError());
}
template <typename S>
void kry_start(lqt_ctx* c, void* V0, const double2* r, const int* src, const double* rn2, int ns) {
    dim3 grid((c->g.V + 255) / 256, ns);
    hipLaunchKernelGGL(k_start<S>, grid, dim3(256), 0, c->stream, (S*)V0, r, src, rn2, c->g.V,
                       sqrt(12.0 * c->g.V));
    LQT_HIP(hipGetLastError());
}

template <typename S>
int kry_carry_blocks(const lqt_ctx* c) {
    return (int)((kry_chunks<S>(c) + 255) / 256);
}
template <typename S>
void kry_sstep_carry(lqt_ctx* c, double2* x, const int* act, void* Kb, long long kstride, int ns, const KryState& st,
                     double theta, double sigma, double* part, double* rn2) {
    const int nblk = kry_carry_blocks<S>(c);
    dim3 grid(nblk, ns);
    hipLaunchKernelGGL(k_sstep_carry<S>, grid, dim3(256), 0, c->stream, x, act, (S*)Kb, kstride, kry_chunks<S>(c), st,
                       theta, sigma, sqrt(12.0 * c->g.V), part);
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_carry_norms, dim3(ns), dim3(256), 0, c->stream, part, nblk, rn2);
    LQT_HIP(hipGetLastError());
}
void kry_start_state_carry(lqt_ctx* c, const KryState& st, const double* target_abs, int ns) {
    hipLaunchKernelGGL(k_start_state_carry, dim3((ns + 63) / 64), dim3(64), 0, c->stream, st, target_abs, ns,
                       sqrt(12.0 * c->g.V));
    LQT_HIP(hipGetLastError());
}

void kry_finish(lqt_ctx* c, const double2* part, int nsb, int j, int ns, const KryState& st, int pass) {
    hipLaunchKernelGGL(k_cgs_finish, dim3(ns), dim3(256), 0, c->stream, part, nsb, j, st, pass, sqrt(12.0 * c->g.V));
    LQT_HIP(hipGetLastError());
}
void kry_norm_givens(lqt_ctx* c, const double* part, int nsb, int j, int ns, const KryState& st) {
    hipLaunchKernelGGL(k_norm_givens, dim3(ns), dim3(64), 0, c->stream, part, nsb, j, st, sqrt(12.0 * c->g.V));
    LQT_HIP(hipGetLastError());
}
void kry_backsolve(lqt_ctx* c, int ns, const KryState& st) {
    hipLaunchKernelGGL(k_backsolve, dim3((ns + 63) / 64), dim3(64), 0, c->stream, st, ns);
    LQT_HIP(hipGetLastError());
}
void kry_start_state(lqt_ctx* c, const KryState& st, const int* src, const double* rn2, const double* target_abs,
                     int ns) {
    hipLaunchKernelGGL(k_start_state, dim3((ns + 63) / 64), dim3(64), 0, c->stream, st, src, rn2, target_abs, ns,
                       sqrt(12.0 * c->g.V));
    LQT_HIP(hipGetLastError());
}

// s-step cycle end: Gram of the ns slots' s+1 stored vectors, then the small solves
constexpr int SGRAM_BLOCKS = 64;
template <typename S>
void sstep_finish(lqt_ctx* c, const void* Vb, long long vstride, int s, int ns, const KryState& st, double theta,
                  double sigma, DBuf& work) {
    const long long n = 12LL * c->g.V;
    const int nv = s + 1;
    const int np = nv * (nv + 1) / 2;
    work.ensure(sizeof(double) * (size_t)ns * SGRAM_BLOCKS * 2 * np);
    double* part = work.as<double>();
    dim3 grid(SGRAM_BLOCKS, ns);
    const double sqrtN = sqrt((double)n);
    c->timer.begin(c->stream, KT_DOTS);
    // up to 9 vectors the vector-ALU pass is faster (measured 1.25 vs 2.4 ms for 9 BF16
    // vectors of 128 probes on 16^3x32); longer 16-bit cycles use the matrix cores
    if (sizeof(S) == 4 && nv > 9) {
        if (nv > 16) throw Error{LQT_EINVAL, "s-step cycles need restart <= 15"};
        if constexpr (sizeof(S) == 4)
            hipLaunchKernelGGL(k_sgram_mf<S>, grid, dim3(256), 0, c->stream, (const S*)Vb, vstride, n, nv, part);
    } else {
#define LQT_SSTEP(NV)                                                                                      \
    case NV:                                                                                               \
        hipLaunchKernelGGL((k_sgram<S, NV>), grid, dim3(256), 0, c->stream, (const S*)Vb, vstride, n, part); \
        break;
    switch (nv) {
        LQT_SSTEP(2)
        LQT_SSTEP(3)
        LQT_SSTEP(4)
        LQT_SSTEP(5)
        LQT_SSTEP(6)
        LQT_SSTEP(7)
        LQT_SSTEP(8)
        LQT_SSTEP(9)
        default: throw Error{LQT_EINVAL, "s-step cycles in FP32/FP64 storage need 1 <= restart <= 8"};
    }
#undef LQT_SSTEP
    }
    LQT_HIP(hipGetLastError());
    c->timer.end(c->stream, (double)nv * n * sizeof(S) * ns);
    c->timer.begin(c->stream, KT_KRYLOV);
#define LQT_SSOLVE(NV)                                                                                           \
    case NV:                                                                                                     \
        hipLaunchKernelGGL(k_sstep_solve_w<NV>, dim3(ns), dim3(64), 0, c->stream, part, SGRAM_BLOCKS, st, theta, sigma, \
                           sqrtN);                                                                               \
        break;
    switch (nv) {
        LQT_SSOLVE(2)
        LQT_SSOLVE(3)
        LQT_SSOLVE(4)
        LQT_SSOLVE(5)
        LQT_SSOLVE(6)
        LQT_SSOLVE(7)
        LQT_SSOLVE(8)
        LQT_SSOLVE(9)
        LQT_SSOLVE(10)
        LQT_SSOLVE(11)
        LQT_SSOLVE(12)
        LQT_SSOLVE(13)
        LQT_SSOLVE(14)
        LQT_SSOLVE(15)
        LQT_SSOLVE(16)
        default: break;
    }
#undef LQT_SSOLVE
    LQT_HIP(hipGetLastError());
    c->timer.end(c->stream);
}

// storage S <-> FP64 over total complex entries (same layout)
template <typename S>
__global__ void k_to_f64(const S* __restrict__ in, double2* __restrict__ out, long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const cx<double> v = ldk<S, double>(in + i);
    out[i] = make_double2(v.x, v.y);
}

template <typename S>
__global__ void k_from_f64(const double2* __restrict__ in, S* __restrict__ out, long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    stk<S, double>(out + i, cx<double>{in[i].x, in[i].y});
}

template <typename S>
void fields_to_f64(lqt_ctx* c, const S* in, double2* out, long long total) {
    if (total <= 0) return;
    hipLaunchKernelGGL(k_to_f64<S>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, in, out, total);
    LQT_HIP(hipGetLastError());
}

template <typename S>
void fields_from_f64(lqt_ctx* c, const double2* in, S* out, long long total) {
    if (total <= 0) return;
    hipLaunchKernelGGL(k_from_f64<S>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, in, out, total);
    LQT_HIP(hipGetLastError());
}

#define INST(S)                                                                                          \
    template void fields_to_f64<S>(lqt_ctx*, const S*, double2*, long long);                             \
    template void fields_from_f64<S>(lqt_ctx*, const double2*, S*, long long);                           \
    template int kry_blocks<S>(const lqt_ctx*);                                                          \
    template int kry_carry_blocks<S>(const lqt_ctx*);                                                    \
    template void kry_dots<S>(lqt_ctx*, const void*, long long, int, int, double2*);                     \
    template void kry_update<S>(lqt_ctx*, void*, long long, int, int, const KryState&, int, double*);    \
    template void kry_xupdate<S>(lqt_ctx*, double2*, const int*, const void*, long long, int,            \
                                 const KryState&);                                                      \
    template void kry_start<S>(lqt_ctx*, void*, const double2*, const int*, const double*, int);        \
    template void kry_sstep_carry<S>(lqt_ctx*, double2*, const int*, void*, long long, int, const KryState&, double, \
                                     double, double*, double*);                                                     \
    template void sstep_finish<S>(lqt_ctx*, const void*, long long, int, int, const KryState&, double, double, \
                                  DBuf&);
INST(double2)
INST(float2)
INST(h2)
INST(b2)

}  // namespace lqt

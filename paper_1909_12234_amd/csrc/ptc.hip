// Gauge-equivariant parallel-transport network used as a right preconditioner.
//
// A field with F features holds F colour 3-vectors per site, laid out like a spinor:
// [rhs][3f + colour][V] (so the 4 spin components of a spinor are its 4 input features).
// Layer l maps F_in -> F_out features:
//   out_f(x) = sum_{p=0..8} sum_g W[p][f][g] (T_p v_g)(x),
//   T_0 = 1, (T_{1+2mu} v)(x) = U_mu(x) v(x+mu), (T_{2+2mu} v)(x) = U_mu(x-mu)^+ v(x-mu),
// with the links of the operator (antiperiodic sign folded in), so the layer commutes with
// gauge transformations.  The adjoint of a layer is a layer with path-swapped (+mu <-> -mu),
// conjugate-transposed weights, which gives the backward pass.  Arithmetic is FP32; the
// weights live on the device in BF16 (rounded once when set).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "blas.h"
#include "gemm.h"
#include "lqt_internal.h"
#include "ptc.h"
#include "solver.h"

namespace lqt {

template <typename S>
__device__ __forceinline__ float2 pld(const S* p) {
    if constexpr (sizeof(S) == 16) {
        double2 v = *(const double2*)p;
        return make_float2((float)v.x, (float)v.y);
    } else {
        return io<S>::ld(p);
    }
}
template <typename S>
__device__ __forceinline__ void pst(S* p, float2 v) {
    if constexpr (sizeof(S) == 16)
        *(double2*)p = make_double2(v.x, v.y);
    else
        io<S>::st(p, v);
}

// One layer, FI -> FO features, one thread per site, nrhs fields (grid.y).  Weights W
// [9][FO][FI] complex FP32 in LDS.  The FP32 links are [mu][ab][V].
template <int FI, int FO, typename SI, typename SO>
__global__ __launch_bounds__(256) void k_ptc_layer(const float2* __restrict__ U, const SI* __restrict__ in,
                                                   SO* __restrict__ out, const float2* __restrict__ Wg, int L0, int L1,
                                                   int L2, int L3) {
    __shared__ float2 W[9 * FO * FI];
    for (int i = threadIdx.x; i < 9 * FO * FI; i += blockDim.x) W[i] = Wg[i];
    __syncthreads();
    const int V = L0 * L1 * L2 * L3;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int r = blockIdx.y;
    const SI* vin = in + (long long)r * FI * 3 * V;
    SO* vout = out + (long long)r * FO * 3 * V;
    const int x = s % L0, y = (s / L0) % L1, z = (s / (L0 * L1)) % L2, t = s / (L0 * L1 * L2);
    const int st[4] = {1, L0, L0 * L1, L0 * L1 * L2};
    const int co[4] = {x, y, z, t};
    const int Ls[4] = {L0, L1, L2, L3};
    float2 acc[FO][3];
#pragma unroll
    for (int f = 0; f < FO; f++)
#pragma unroll
        for (int a = 0; a < 3; a++) acc[f][a] = make_float2(0, 0);
#pragma unroll 1
    for (int p = 0; p < 9; p++) {
        float2 tv[FI][3];
        if (p == 0) {
#pragma unroll
            for (int g = 0; g < FI; g++)
#pragma unroll
                for (int a = 0; a < 3; a++) tv[g][a] = pld<SI>(vin + (long long)(3 * g + a) * V + s);
        } else {
            const int mu = (p - 1) >> 1;
            const bool fwd = ((p - 1) & 1) == 0;
            int ns;
            if (fwd)
                ns = (co[mu] == Ls[mu] - 1) ? s - (Ls[mu] - 1) * st[mu] : s + st[mu];
            else
                ns = (co[mu] == 0) ? s + (Ls[mu] - 1) * st[mu] : s - st[mu];
            const int ls = fwd ? s : ns;
            float2 u[9];
#pragma unroll
            for (int i = 0; i < 9; i++) u[i] = U[(long long)(mu * 9 + i) * V + ls];
#pragma unroll
            for (int g = 0; g < FI; g++) {
                float2 v[3];
#pragma unroll
                for (int b = 0; b < 3; b++) v[b] = pld<SI>(vin + (long long)(3 * g + b) * V + ns);
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    float re = 0, im = 0;
#pragma unroll
                    for (int b = 0; b < 3; b++) {
                        // forward: U[a][b]; backward: conj(U[b][a])
                        const float2 l = fwd ? u[3 * a + b] : make_float2(u[3 * b + a].x, -u[3 * b + a].y);
                        re += l.x * v[b].x - l.y * v[b].y;
                        im += l.x * v[b].y + l.y * v[b].x;
                    }
                    tv[g][a] = make_float2(re, im);
                }
            }
        }
#pragma unroll
        for (int f = 0; f < FO; f++)
#pragma unroll
            for (int g = 0; g < FI; g++) {
                const float2 w = W[(p * FO + f) * FI + g];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    acc[f][a].x += w.x * tv[g][a].x - w.y * tv[g][a].y;
                    acc[f][a].y += w.x * tv[g][a].y + w.y * tv[g][a].x;
                }
            }
    }
#pragma unroll
    for (int f = 0; f < FO; f++)
#pragma unroll
        for (int a = 0; a < 3; a++) pst<SO>(vout + (long long)(3 * f + a) * V + s, acc[f][a]);
}

// Transport only, all nine paths: out[p][g] = T_p in_g (FP64 fields [g][colour][V] in,
// [p][g][colour][V] out; grid (site blocks, F, 9)), used for the weight gradients.
__global__ __launch_bounds__(256) void k_transport9(const double2* __restrict__ U, const double2* __restrict__ in,
                                                    double2* __restrict__ out, int F, int L0, int L1, int L2, int L3) {
    const int V = L0 * L1 * L2 * L3;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const int g = blockIdx.y, p = blockIdx.z;
    const int x = s % L0, y = (s / L0) % L1, z = (s / (L0 * L1)) % L2, t = s / (L0 * L1 * L2);
    const int st[4] = {1, L0, L0 * L1, L0 * L1 * L2};
    const int co[4] = {x, y, z, t};
    const int Ls[4] = {L0, L1, L2, L3};
    const double2* vin = in + (long long)3 * g * V;
    double2* vo = out + ((long long)p * F + g) * 3 * V;
    if (p == 0) {
        for (int a = 0; a < 3; a++) vo[(long long)a * V + s] = vin[(long long)a * V + s];
        return;
    }
    const int mu = (p - 1) >> 1;
    const bool fwd = ((p - 1) & 1) == 0;
    int ns;
    if (fwd)
        ns = (co[mu] == Ls[mu] - 1) ? s - (Ls[mu] - 1) * st[mu] : s + st[mu];
    else
        ns = (co[mu] == 0) ? s + (Ls[mu] - 1) * st[mu] : s - st[mu];
    const int ls = fwd ? s : ns;
    double2 u[9], v[3];
    for (int i = 0; i < 9; i++) u[i] = U[(long long)(mu * 9 + i) * V + ls];
    for (int b = 0; b < 3; b++) v[b] = vin[(long long)b * V + ns];
    for (int a = 0; a < 3; a++) {
        double re = 0, im = 0;
        for (int b = 0; b < 3; b++) {
            const double2 l = fwd ? u[3 * a + b] : make_double2(u[3 * b + a].x, -u[3 * b + a].y);
            re += l.x * v[b].x - l.y * v[b].y;
            im += l.x * v[b].y + l.y * v[b].x;
        }
        vo[(long long)a * V + s] = make_double2(re, im);
    }
}

// delta = (a - e) * wq[q] for pair q (grid (256, np)); part[q*256 + b] = partial |a - e|^2
__global__ __launch_bounds__(256) void k_ptc_delta(const double2* __restrict__ a, const double2* __restrict__ e,
                                                   const double* __restrict__ wq, long long n,
                                                   double2* __restrict__ del, double* __restrict__ part) {
    __shared__ double red[256];
    const int q = blockIdx.y;
    const double w = wq[q];
    double acc = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double2 av = a[q * n + i], ev = e[q * n + i];
        const double dx = av.x - ev.x, dy = av.y - ev.y;
        acc += dx * dx + dy * dy;
        del[q * n + i] = make_double2(dx * w, dy * w);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)q * gridDim.x + blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- host side
// four layers, 12 -> 24 -> 24 -> 24 -> 12 complex channels (4 -> 8 -> 8 -> 8 -> 4 features)
const int FEATS[5] = {4, 8, 8, 8, 4};

int ptc_weight_count() {
    int n = 0;
    for (int l = 0; l < NL; l++) n += 9 * FEATS[l] * FEATS[l + 1];
    return n;  // complex entries
}

static float bf16_round(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

void ptc_set(lqt_ctx* c, const float* w, bool round_bf16) {
    const int nw = ptc_weight_count();
    c->net.w.assign(w, w + 2 * nw);
    std::vector<float> dev(2 * nw);
    for (int i = 0; i < 2 * nw; i++) dev[i] = round_bf16 ? bf16_round(w[i]) : w[i];
    c->net.wf.ensure(sizeof(float) * 2 * nw);
    LQT_HIP(hipMemcpyAsync(c->net.wf.p, dev.data(), sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    c->net.set = true;
}

template <int FI, int FO, typename SI, typename SO>
static void layer_launch(lqt_ctx* c, const float2* W, const SI* in, SO* out, int nrhs) {
    const Geom& g = c->g;
    dim3 grid((g.V + 255) / 256, nrhs);
    hipLaunchKernelGGL((k_ptc_layer<FI, FO, SI, SO>), grid, dim3(256), 0, c->stream, c->U[LQT_F32].as<float2>(), in,
                       out, W, g.L[0], g.L[1], g.L[2], g.L[3]);
    LQT_HIP(hipGetLastError());
}

template <typename S>
void ptc_apply(lqt_ctx* c, const S* in, S* out, int nrhs) {
    if (nrhs <= 0) return;
    const long long V = c->g.V;
    c->net.act.ensure(sizeof(float2) * (size_t)nrhs * 24 * V * 2);
    float2* a = c->net.act.as<float2>();
    float2* b = a + (size_t)nrhs * 24 * V;
    const float2* W = c->net.wf.as<float2>();
    c->timer.begin(c->stream, KT_NET);
    layer_launch<4, 8, S, float2>(c, W, in, a, nrhs);
    W += 9 * 4 * 8;
    layer_launch<8, 8, float2, float2>(c, W, a, b, nrhs);
    W += 9 * 8 * 8;
    layer_launch<8, 8, float2, float2>(c, W, b, a, nrhs);
    W += 9 * 8 * 8;
    layer_launch<8, 4, float2, S>(c, W, a, out, nrhs);
    // algorithmic bytes: input, output and the two intermediate FP32 fields, links per layer
    c->timer.end(c->stream, (double)V * nrhs * (12.0 * sizeof(S) * 2 + 24.0 * 8 * 4) + 4.0 * 72 * 4 * V);
}

template void ptc_apply<double2>(lqt_ctx*, const double2*, double2*, int);
template void ptc_apply<float2>(lqt_ctx*, const float2*, float2*, int);
template void ptc_apply<h2>(lqt_ctx*, const h2*, h2*, int);
template void ptc_apply<b2>(lqt_ctx*, const b2*, b2*, int);

// ---------------------------------------------------------------- training
// One FP64-activation pass: forward with stored activations, loss, backward through the
// adjoint layers and weight gradients G_l[p][f][g] = sum_x conj(T_p a_{l-1,g}) delta_{l,f}.

template <int FI, int FO>
static void layer64(lqt_ctx* c, const float2* W, const double2* in, double2* out, int nrhs) {
    layer_launch<FI, FO, double2, double2>(c, W, in, out, nrhs);
}

static void layer64_dyn(lqt_ctx* c, int fi, int fo, const float2* W, const double2* in, double2* out, int nrhs) {
    if (fi == 4 && fo == 8) layer64<4, 8>(c, W, in, out, nrhs);
    else if (fi == 8 && fo == 8) layer64<8, 8>(c, W, in, out, nrhs);
    else if (fi == 8 && fo == 4) layer64<8, 4>(c, W, in, out, nrhs);
    else throw Error{LQT_EINVAL, "unsupported layer shape"};
}

// adjoint weights: W'[p'][g][f] = conj(W[p][f][g]), p' = path with the opposite direction
static std::vector<float> adjoint_weights(const float* W, int fi, int fo) {
    std::vector<float> A(2 * 9 * fi * fo);
    for (int p = 0; p < 9; p++) {
        const int pa = (p == 0) ? 0 : (((p - 1) & 1) ? p - 1 : p + 1);
        for (int f = 0; f < fo; f++)
            for (int g = 0; g < fi; g++) {
                const float* w = W + 2 * ((p * fo + f) * fi + g);
                float* o = A.data() + 2 * ((pa * fi + g) * fo + f);
                o[0] = w[0];
                o[1] = -w[1];
            }
    }
    return A;
}

// Loss sum_pairs ||M r - e||^2 / ||e||^2 and its gradient with respect to conj(W) (FP64
// fields r, e: np spinors in device layout).  grad receives 2 * ptc_weight_count() doubles.
// Forward with stored activations a_1..a_4; delta_4 = (a_4 - e)/||e||^2; delta_{l-1} =
// L_l^+ delta_l (the adjoint layer); G_l[p][f][g] = sum_x conj(T_p a_{l-1,g}) . delta_{l,f}
// from one FP64 MFMA Gram product per (layer, pair); one device-to-host copy per call.
double ptc_loss_grad(lqt_ctx* c, const double2* r, const double2* e, int np, const float* Wh, std::vector<double>& grad,
                     const std::vector<double>& enorm2) {
    const long long V = c->g.V;
    const long long n = 12 * V;
    const int nw = ptc_weight_count();
    grad.assign(2 * nw, 0.0);
    DBuf* tw = c->net.train;  // workspace kept across calls
    // weights of this pass and their adjoints
    std::vector<float> adj;
    int woff[NL];
    for (int l = 0, off = 0; l < NL; l++) {
        woff[l] = off;
        std::vector<float> a = adjoint_weights(Wh + 2 * off, FEATS[l], FEATS[l + 1]);
        adj.insert(adj.end(), a.begin(), a.end());
        off += 9 * FEATS[l] * FEATS[l + 1];
    }
    tw[0].ensure(sizeof(float) * 2 * nw);
    tw[1].ensure(sizeof(float) * 2 * nw);
    LQT_HIP(hipMemcpyAsync(tw[0].p, Wh, sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    LQT_HIP(hipMemcpyAsync(tw[1].p, adj.data(), sizeof(float) * 2 * nw, hipMemcpyHostToDevice, c->stream));
    // activations a_1..a_4 (FP64, [pair][3F][V]) in one buffer, two delta buffers, the
    // transported inputs of one pair, the Gram blocks of every (layer, pair), small vectors
    size_t aoff[NL + 2];
    aoff[1] = 0;
    for (int l = 1; l <= NL; l++) aoff[l + 1] = aoff[l] + (size_t)np * 3 * FEATS[l] * V;
    tw[2].ensure(sizeof(double2) * aoff[NL + 1]);
    tw[3].ensure(sizeof(double2) * (size_t)np * 24 * V);
    tw[4].ensure(sizeof(double2) * (size_t)np * 24 * V);
    tw[5].ensure(sizeof(double2) * (size_t)9 * 8 * 3 * V);
    tw[6].ensure(sizeof(double2) * (size_t)np * nw);
    const int nbl = 256;
    tw[7].ensure(sizeof(double) * ((size_t)np * nbl + np));
    auto act = [&](int l) { return tw[2].as<double2>() + aoff[l]; };
    double2* G = tw[6].as<double2>();
    double* lpart = tw[7].as<double>();
    double* wq = lpart + (size_t)np * nbl;
    std::vector<double> hw(np);
    for (int q = 0; q < np; q++) hw[q] = 1.0 / enorm2[q];
    LQT_HIP(hipMemcpyAsync(wq, hw.data(), sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
    const float2* Wd = tw[0].as<float2>();
    const float2* Wa = tw[1].as<float2>();
    const double2* a_prev = r;
    for (int l = 0; l < NL; l++) {
        layer64_dyn(c, FEATS[l], FEATS[l + 1], Wd + woff[l], a_prev, act(l + 1), np);
        a_prev = act(l + 1);
    }
    hipLaunchKernelGGL(k_ptc_delta, dim3(nbl, np), dim3(256), 0, c->stream, act(NL), e, wq, n,
                       tw[3].as<double2>(), lpart);
    LQT_HIP(hipGetLastError());
    int cur = 3;
    for (int l = NL; l >= 1; l--) {
        const int fi = FEATS[l - 1], fo = FEATS[l];
        const double2* ain = (l == 1) ? r : act(l - 1);
        const double2* dl = tw[cur].as<double2>();
        for (int q = 0; q < np; q++) {
            dim3 grid((unsigned)((V + 255) / 256), fi, 9);
            hipLaunchKernelGGL(k_transport9, grid, dim3(256), 0, c->stream, c->U[LQT_F64].as<double2>(),
                               ain + (size_t)q * 3 * fi * V, tw[5].as<double2>(), fi, c->g.L[0], c->g.L[1],
                               c->g.L[2], c->g.L[3]);
            LQT_HIP(hipGetLastError());
            // C[p*fi + g][f] = sum_x conj(T_p a_g) . delta_f   (vectors of length 3V)
            gemm_gram(c, tw[5].as<double2>(), 9 * fi, dl + (size_t)q * 3 * fo * V, fo,
                      G + (size_t)q * nw + woff[l - 1], 3LL * V);
        }
        if (l > 1) {  // delta_{l-1} = L_l^+ delta_l
            const int nxt = (cur == 3) ? 4 : 3;
            layer64_dyn(c, fo, fi, Wa + woff[l - 1], dl, tw[nxt].as<double2>(), np);
            cur = nxt;
        }
    }
    std::vector<double2> hG((size_t)np * nw);
    std::vector<double> hl((size_t)np * nbl);
    LQT_HIP(hipMemcpyAsync(hG.data(), G, sizeof(double2) * hG.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipMemcpyAsync(hl.data(), lpart, sizeof(double) * hl.size(), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    double loss = 0;
    for (int q = 0; q < np; q++) {
        double lq = 0;
        for (int b = 0; b < nbl; b++) lq += hl[(size_t)q * nbl + b];
        loss += lq * hw[q];
    }
    for (int q = 0; q < np; q++)
        for (int l = 0; l < NL; l++) {
            const int fi = FEATS[l], fo = FEATS[l + 1];
            const double2* Gq = hG.data() + (size_t)q * nw + woff[l];
            for (int p = 0; p < 9; p++)
                for (int g = 0; g < fi; g++)
                    for (int f = 0; f < fo; f++) {
                        const double2 v = Gq[(p * fi + g) * fo + f];
                        double* gw = grad.data() + 2 * (woff[l] + (p * fo + f) * fi + g);
                        gw[0] += v.x;
                        gw[1] += v.y;
                    }
        }
    return loss;
}

// r = A e (FP64) for np error fields e (device layout), then the summed loss and gradient.
double ptc_pairs_loss_grad(lqt_ctx* c, const double2* e, double2* r, int np, const float* Wh,
                           std::vector<double>& grad) {
    const long long n = 12LL * c->g.V;
    dslash(c, LQT_F64, LQT_A, e, r, np, n, n);
    c->scratch[9].ensure(sizeof(double) * np);
    std::vector<double> en(np);
    norm2_fields(c, e, np, c->scratch[9].as<double>());
    LQT_HIP(hipMemcpyAsync(en.data(), c->scratch[9].p, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    for (int q = 0; q < np; q++) LQT_CHECK(en[q] > 0, LQT_EINVAL, "an error field is zero");
    return ptc_loss_grad(c, r, e, np, Wh, grad, en);
}

}  // namespace lqt

namespace {

template <typename F>
int guard(lqt_ctx* c, F&& f) {
    try {
        f();
        return LQT_OK;
    } catch (const lqt::Error& e) {
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

}  // namespace

extern "C" {

int lqt_precond_set(lqt_ctx* c, const void* w, size_t nbytes) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(w && nbytes == sizeof(float) * 2 * (size_t)lqt::ptc_weight_count(), LQT_EINVAL,
                  "weights must be " + std::to_string(8 * lqt::ptc_weight_count()) + " bytes of complex FP32");
        const float* f = (const float*)w;
        for (int i = 0; i < 2 * lqt::ptc_weight_count(); i++) LQT_CHECK(std::isfinite(f[i]), LQT_ENAN, "weight is NaN");
        lqt::ptc_set(c, f, true);
    });
}

int lqt_precond_get(lqt_ctx* c, void* w, size_t nbytes) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(w && nbytes == sizeof(float) * c->net.w.size(), LQT_EINVAL, "bad weight buffer");
        std::memcpy(w, c->net.w.data(), nbytes);
    });
}

int lqt_precond_apply(lqt_ctx* c, const double* in, double* out, int nrhs) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(nrhs >= 0 && (nrhs == 0 || (in && out)), LQT_EINVAL, "bad fields");
        if (nrhs == 0) return;
        const long long n = 12LL * c->g.V;
        lqt::DBuf a, b;
        a.ensure(sizeof(double2) * (size_t)nrhs * n);
        b.ensure(sizeof(double2) * (size_t)nrhs * n);
        lqt::to_device_layout(c, (const double2*)in, a.as<double2>(), nrhs);
        lqt::ptc_apply<double2>(c, a.as<double2>(), b.as<double2>(), nrhs);
        lqt::from_device_layout(c, b.as<double2>(), (double2*)out, nrhs);
        LQT_HIP(hipStreamSynchronize(c->stream));
    });
}

int lqt_precond_loss_grad(lqt_ctx* c, const double* e, int npairs, double* loss, double* grad) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(c->net.set, LQT_ESTATE, "no preconditioner weights");
        LQT_CHECK(npairs >= 1 && e && loss && grad, LQT_EINVAL, "bad arguments");
        const long long n = 12LL * c->g.V;
        const int nw = lqt::ptc_weight_count();
        const int chunk = 4;
        lqt::DBuf E, R;
        E.ensure(sizeof(double2) * (size_t)chunk * n);
        R.ensure(sizeof(double2) * (size_t)chunk * n);
        std::vector<double> gsum(2 * nw, 0.0), g;
        double lsum = 0;
        for (int p0 = 0; p0 < npairs; p0 += chunk) {
            const int np = std::min(chunk, npairs - p0);
            lqt::to_device_layout(c, (const double2*)e + (size_t)p0 * n, E.as<double2>(), np);
            lsum += lqt::ptc_pairs_loss_grad(c, E.as<double2>(), R.as<double2>(), np, c->net.w.data(), g);
            for (int i = 0; i < 2 * nw; i++) gsum[i] += g[i];
        }
        *loss = lsum / npairs;
        for (int i = 0; i < 2 * nw; i++) grad[i] = gsum[i] / npairs;
    });
}

int lqt_precond_train(lqt_ctx* c, int npairs, uint64_t seed, const lqt_train_opts* opts, double* final_loss) {
    if (!c) return LQT_EINVAL;
    return guard(c, [&] {
        LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "not available for a context of several lattices");
        LQT_CHECK(c->have_gauge, LQT_ESTATE, "no gauge field set (call lqt_set_gauge)");
        LQT_CHECK(npairs >= 1, LQT_EINVAL, "npairs must be >= 1");
        LQT_CHECK(!opts || (opts->epochs >= 0 && opts->batch >= 0 && opts->lr >= 0 && opts->pair_xi >= 0 &&
                            opts->pair_xi < 1),
                  LQT_EINVAL, "bad options");
        const int epochs = (opts && opts->epochs > 0) ? opts->epochs : 4;
        const double lr = (opts && opts->lr > 0) ? opts->lr : 1e-3;
        const int batch = (opts && opts->batch > 0) ? opts->batch : 4;  // pairs per optimiser step
        const double pair_xi = opts ? opts->pair_xi : 0.0;
        const int nw = lqt::ptc_weight_count();
        const long long n = 12LL * c->g.V;
        // the training set stays resident: npairs error fields e (FP64)
        size_t fr = 0, tot = 0;
        LQT_HIP(hipMemGetInfo(&fr, &tot));
        const size_t need = sizeof(double2) * (size_t)npairs * n;
        LQT_CHECK(need <= fr / 2, LQT_ENOMEM, "training set does not fit in half of the free device memory");
        lqt::DBuf E, R, G;
        E.ensure(need);
        R.ensure(sizeof(double2) * (size_t)batch * n);
        // errors: Gaussian g, or the solver's own output e = A^{-1}_{pair_xi} g (r = A e exactly)
        const int gchunk = 16;
        if (pair_xi > 0) G.ensure(sizeof(double2) * (size_t)gchunk * n);
        for (int p0 = 0; p0 < npairs; p0 += gchunk) {
            const int np = std::min(gchunk, npairs - p0);
            double2* Ep = E.as<double2>() + (size_t)p0 * n;
            const uint64_t s0 = seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(p0 + 1));
            if (pair_xi > 0) {
                lqt::gaussian_fields(c, s0, n, np, G.as<double2>());
                lqt::SolveOpts so;
                so.prec = LQT_F32;
                lqt::solve_fields(c, G.as<double2>(), Ep, np, pair_xi, so, nullptr);
            } else {
                lqt::gaussian_fields(c, s0, n, np, Ep);
            }
        }
        // start: the identity scaled by |4+m|^{-1/4} per layer (M = 1/(4+m)) unless set
        std::vector<float> W(2 * nw, 0.0f);
        if (c->net.set) {
            W = c->net.w;
        } else {
            const float s = (float)std::pow(1.0 / std::fabs(4.0 + c->mass), 0.25);
            for (int l = 0, off = 0; l < lqt::NL; l++) {
                const int fi = lqt::FEATS[l], fo = lqt::FEATS[l + 1];
                for (int f = 0; f < std::min(fi, fo); f++) W[2 * (off + f * fi + f)] = s;  // p = 0
                off += 9 * fi * fo;
            }
        }
        std::vector<double> m1(2 * nw, 0.0), m2(2 * nw, 0.0), grad;
        const double b1 = 0.9, b2 = 0.999, eps = 1e-12;
        double loss = 0;
        long long t = 0;
        for (int ep = 0; ep < epochs; ep++) {
            double eloss = 0;
            for (int p0 = 0; p0 < npairs; p0 += batch) {
                const int np = std::min(batch, npairs - p0);
                eloss += lqt::ptc_pairs_loss_grad(c, E.as<double2>() + (size_t)p0 * n, R.as<double2>(), np,
                                                  W.data(), grad);
                t++;
                for (int i = 0; i < 2 * nw; i++) {  // Adam on the real and imaginary parts
                    const double gi = grad[i] / np;
                    m1[i] = b1 * m1[i] + (1 - b1) * gi;
                    m2[i] = b2 * m2[i] + (1 - b2) * gi * gi;
                    const double mh = m1[i] / (1 - std::pow(b1, (double)t)), vh = m2[i] / (1 - std::pow(b2, (double)t));
                    W[i] -= (float)(lr * mh / (std::sqrt(vh) + eps));
                }
            }
            loss = eloss / npairs;
            if (opts && opts->verbose) {
                fprintf(stderr, "[lqtrace] train epoch %d: mean loss %.5e\n", ep, loss);
                fflush(stderr);
            }
        }
        lqt::ptc_set(c, W.data(), true);
        if (final_loss) *final_loss = loss;
    });
}

}  // extern "C"

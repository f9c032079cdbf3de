// Layout kernels: canonical AoS complex128 <-> device SoA fields, gauge ingest with the
// unitarity check and precision copies.
#include "lqt_internal.h"

namespace lqt {

// One thread per link: check U^+U = 1 and det U = 1, fold the antiperiodic sign into the
// last time slice, scatter into [mu][ab][V] for every storage precision.
__global__ void k_gauge_ingest(const double2* __restrict__ canon, int V, int slice, int Lt, int antiperiodic,
                               double2* __restrict__ u64, float2* __restrict__ u32, h2* __restrict__ u16,
                               b2* __restrict__ ubf, double* __restrict__ err_unit, double* __restrict__ err_det) {
    __shared__ double s_u[256], s_d[256];
    int tid = threadIdx.x;
    long long idx = (long long)blockIdx.x * blockDim.x + tid;  // link index = site*4 + mu
    double eu = 0, ed = 0;
    if (idx < 4LL * V) {
        int site = (int)(idx >> 2), mu = (int)(idx & 3);
        double2 m[9];
        for (int i = 0; i < 9; i++) m[i] = canon[idx * 9 + i];
        // U^+ U - 1
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double re = 0, im = 0;
                for (int k = 0; k < 3; k++) {
                    double2 p = m[3 * k + a], q = m[3 * k + b];  // conj(U_ka) U_kb
                    re += p.x * q.x + p.y * q.y;
                    im += p.x * q.y - p.y * q.x;
                }
                if (a == b) re -= 1.0;
                eu = fmax(eu, sqrt(re * re + im * im));
            }
        // determinant by cofactor expansion along the first row
        auto mul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
        auto sub = [](double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); };
        double2 c0 = sub(mul(m[4], m[8]), mul(m[5], m[7]));
        double2 c1 = sub(mul(m[3], m[8]), mul(m[5], m[6]));
        double2 c2 = sub(mul(m[3], m[7]), mul(m[4], m[6]));
        double2 d = sub(mul(m[0], c0), mul(m[1], c1));
        double2 t2 = mul(m[2], c2);
        d.x += t2.x;
        d.y += t2.y;
        ed = sqrt((d.x - 1.0) * (d.x - 1.0) + d.y * d.y);
        if (!(eu == eu) || !(ed == ed)) eu = ed = 1e300;  // NaN -> reject
        double sgn = (antiperiodic && (site / slice) == Lt - 1 && mu == 3) ? -1.0 : 1.0;
        for (int i = 0; i < 9; i++) {
            double2 v = make_double2(sgn * m[i].x, sgn * m[i].y);
            long long o = (long long)(mu * 9 + i) * V + site;
            u64[o] = v;
            float2 f = make_float2((float)v.x, (float)v.y);
            u32[o] = f;
            io<h2>::st(u16 + o, f);
            io<b2>::st(ubf + o, f);
        }
    }
    s_u[tid] = eu;
    s_d[tid] = ed;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) {
            s_u[tid] = fmax(s_u[tid], s_u[tid + w]);
            s_d[tid] = fmax(s_d[tid], s_d[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        err_unit[blockIdx.x] = s_u[0];
        err_det[blockIdx.x] = s_d[0];
    }
}

void gauge_upload(lqt_ctx* c, const double* links, int on_device, double* max_unit_err, double* max_det_err) {
    const int V = c->g.V;
    const size_t nlink = 4ull * V * 9;
    DBuf staging;
    const double2* src = (const double2*)links;
    if (!on_device) {
        staging.ensure(nlink * sizeof(double2));
        LQT_HIP(hipMemcpyAsync(staging.p, links, nlink * sizeof(double2), hipMemcpyHostToDevice, c->stream));
        src = staging.as<double2>();
    }
    c->U[LQT_F64].ensure(nlink * sizeof(double2));
    c->U[LQT_F32].ensure(nlink * sizeof(float2));
    c->U[LQT_F16].ensure(nlink * sizeof(h2));
    c->U[LQT_BF16].ensure(nlink * sizeof(b2));
    const int bs = 256;
    const int nb = (int)((4LL * V + bs - 1) / bs);
    DBuf errs;
    errs.ensure(2ull * nb * sizeof(double));
    int slice = c->g.L[0] * c->g.L[1] * c->g.L[2];
    hipLaunchKernelGGL(k_gauge_ingest, dim3(nb), dim3(bs), 0, c->stream, src, V, slice, c->g.L[3], c->antiperiodic,
                       c->U[LQT_F64].as<double2>(), c->U[LQT_F32].as<float2>(), c->U[LQT_F16].as<h2>(),
                       c->U[LQT_BF16].as<b2>(), errs.as<double>(), errs.as<double>() + nb);
    LQT_HIP(hipGetLastError());
    std::vector<double> h(2ull * nb);
    LQT_HIP(hipMemcpyAsync(h.data(), errs.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    double mu = 0, md = 0;
    for (int i = 0; i < nb; i++) {
        mu = fmax(mu, h[i]);
        md = fmax(md, h[nb + i]);
    }
    *max_unit_err = mu;
    *max_det_err = md;
}

// canonical [rhs][site][12] <-> device [rhs][12][site]; one thread per (site, comp) of one
// rhs, reading the canonical side in order (consecutive threads = consecutive components).
__global__ void k_aos_to_soa(const double2* __restrict__ in, double2* __restrict__ out, int V, int nrhs) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long n = 12LL * V;
    if (i >= n * nrhs) return;
    long long r = i / n, e = i - r * n;
    int site = (int)(e / 12), comp = (int)(e - 12LL * site);
    out[r * n + (long long)comp * V + site] = in[i];
}

__global__ void k_soa_to_aos(const double2* __restrict__ in, double2* __restrict__ out, int V, int nrhs) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long n = 12LL * V;
    if (i >= n * nrhs) return;
    long long r = i / n, e = i - r * n;
    int site = (int)(e / 12), comp = (int)(e - 12LL * site);
    out[i] = in[r * n + (long long)comp * V + site];
}

// float2 <-> storage conversions (FP32 canonical input for the reduced-precision applies)
template <typename SO>
__global__ void k_c64_to_soa(const float2* __restrict__ in, SO* __restrict__ out, int V, int nrhs) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long n = 12LL * V;
    if (i >= n * nrhs) return;
    long long r = i / n, e = i - r * n;
    int site = (int)(e / 12), comp = (int)(e - 12LL * site);
    io<SO>::st(out + r * n + (long long)comp * V + site, in[i]);
}
template <typename SI>
__global__ void k_soa_to_c64(const SI* __restrict__ in, float2* __restrict__ out, int V, int nrhs) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long n = 12LL * V;
    if (i >= n * nrhs) return;
    long long r = i / n, e = i - r * n;
    int site = (int)(e / 12), comp = (int)(e - 12LL * site);
    out[i] = io<SI>::ld(in + r * n + (long long)comp * V + site);
}

static inline dim3 grid_for(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

void to_device_layout(lqt_ctx* c, const double2* canon, double2* dev, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL(k_aos_to_soa, grid_for(n, 256), dim3(256), 0, c->stream, canon, dev, c->g.V,
                       nrhs);
    LQT_HIP(hipGetLastError());
}
void from_device_layout(lqt_ctx* c, const double2* dev, double2* canon, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL(k_soa_to_aos, grid_for(n, 256), dim3(256), 0, c->stream, dev, canon, c->g.V,
                       nrhs);
    LQT_HIP(hipGetLastError());
}

template <typename S>
void convert_in_c64(lqt_ctx* c, const float2* canon, S* dev, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL(k_c64_to_soa<S>, grid_for(n, 256), dim3(256), 0, c->stream, canon, dev, c->g.V, nrhs);
    LQT_HIP(hipGetLastError());
}
template <typename S>
void convert_out_c64(lqt_ctx* c, const S* dev, float2* canon, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL(k_soa_to_c64<S>, grid_for(n, 256), dim3(256), 0, c->stream, dev, canon, c->g.V, nrhs);
    LQT_HIP(hipGetLastError());
}

template void convert_in_c64<float2>(lqt_ctx*, const float2*, float2*, int);
template void convert_in_c64<h2>(lqt_ctx*, const float2*, h2*, int);
template void convert_in_c64<b2>(lqt_ctx*, const float2*, b2*, int);
template void convert_out_c64<float2>(lqt_ctx*, const float2*, float2*, int);
template void convert_out_c64<h2>(lqt_ctx*, const h2*, float2*, int);
template void convert_out_c64<b2>(lqt_ctx*, const b2*, float2*, int);

}  // namespace lqt

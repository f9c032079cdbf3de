// Layout kernels: canonical AoS complex128 <-> device SoA fields, gauge ingest with the
// unitarity check and precision copies.
#include "lqt_internal.h"

namespace lqt {

// One thread per link of the canonical field (lattices one after the other, each
// [site][mu][a][b]): check U^+U = 1 and det U = 1, fold the antiperiodic sign into the last
// time slice of its lattice, scatter into [mu][ab][V] at the lattice's device sites for
// every storage precision (FP32 and FP16 rounded from FP64, BF16 from the FP32 value).
__global__ void k_gauge_ingest(const double2* __restrict__ canon, LatTab t, long long nlinks, int antiperiodic,
                               double2* __restrict__ u64, float2* __restrict__ u32, h2* __restrict__ u16,
                               b2* __restrict__ ubf, double* __restrict__ err_unit, double* __restrict__ err_det) {
    __shared__ double s_u[256], s_d[256];
    int tid = threadIdx.x;
    long long idx = (long long)blockIdx.x * blockDim.x + tid;  // link index = canonical site*4 + mu
    double eu = 0, ed = 0;
    if (idx < nlinks) {
        const int csite = (int)(idx >> 2), mu = (int)(idx & 3);
        int k = 0;
        for (int i = 1; i < t.nlat; i++)
            if (csite >= t.coff[i]) k = i;
        const int sl = csite - t.coff[k];
        const int V = t.off[t.nlat];
        const int site = t.off[k] + sl;
        const int Lt = t.L[k][3], slice = t.L[k][0] * t.L[k][1] * t.L[k][2];
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
        double sgn = (antiperiodic && (sl / slice) == Lt - 1 && mu == 3) ? -1.0 : 1.0;
        for (int i = 0; i < 9; i++) {
            double2 v = make_double2(sgn * m[i].x, sgn * m[i].y);
            long long o = (long long)(mu * 9 + i) * V + site;
            u64[o] = v;
            float2 f = make_float2((float)v.x, (float)v.y);
            u32[o] = f;
            // FP16: rounded once from FP64 (to nearest even); BF16: from the FP32 value
            h2 hv;
            hv.x = __half_raw{static_cast<_Float16>(v.x)};
            hv.y = __half_raw{static_cast<_Float16>(v.y)};
            u16[o] = hv;
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
    const long long nlinks = 4LL * c->g.canon_sites;  // canonical links (no padding)
    const size_t ncanon = (size_t)nlinks * 9;
    const size_t ndev = 36ull * V;
    DBuf staging;
    const double2* src = (const double2*)links;
    if (!on_device) {
        staging.ensure(ncanon * sizeof(double2));
        LQT_HIP(hipMemcpyAsync(staging.p, links, ncanon * sizeof(double2), hipMemcpyHostToDevice, c->stream));
        src = staging.as<double2>();
    }
    c->U[LQT_F64].ensure(ndev * sizeof(double2));
    c->U[LQT_F32].ensure(ndev * sizeof(float2));
    c->U[LQT_F16].ensure(ndev * sizeof(h2));
    c->U[LQT_BF16].ensure(ndev * sizeof(b2));
    if (c->g.lat.nlat > 1) {  // padding sites between lattices hold zero links
        LQT_HIP(hipMemsetAsync(c->U[LQT_F64].p, 0, ndev * sizeof(double2), c->stream));
        LQT_HIP(hipMemsetAsync(c->U[LQT_F32].p, 0, ndev * sizeof(float2), c->stream));
        LQT_HIP(hipMemsetAsync(c->U[LQT_F16].p, 0, ndev * sizeof(h2), c->stream));
        LQT_HIP(hipMemsetAsync(c->U[LQT_BF16].p, 0, ndev * sizeof(b2), c->stream));
    }
    const int bs = 256;
    const int nb = (int)((nlinks + bs - 1) / bs);
    DBuf errs;
    errs.ensure(2ull * nb * sizeof(double));
    hipLaunchKernelGGL(k_gauge_ingest, dim3(nb), dim3(bs), 0, c->stream, src, c->g.lat, nlinks, c->antiperiodic,
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

// canonical [rhs][lattice][site][12] <-> device [rhs][12][site] (lattice k at device sites
// off[k]..); one thread per device element, consecutive threads = consecutive sites of one
// component.  Padding sites are written as zeros on the way in and skipped on the way out.
template <typename SI, typename SO>
__global__ void k_to_dev(const SI* __restrict__ in, SO* __restrict__ out, LatTab t, long long ncanon, int nrhs) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long V = t.off[t.nlat], n = 12 * V;
    if (i >= n * nrhs) return;
    const long long r = i / n, e = i - r * n;
    const int comp = (int)(e / V);
    const uint32_t s = (uint32_t)(e - comp * V);
    int k;
    uint32_t sl;
    const bool ok = lat_site(t, s, k, sl);
    if constexpr (sizeof(SI) == 16 && sizeof(SO) == 16) {
        out[i] = ok ? in[r * ncanon + 12LL * (t.coff[k] + sl) + comp] : make_double2(0, 0);
    } else {
        const float2 v = ok ? in[r * ncanon + 12LL * (t.coff[k] + sl) + comp] : make_float2(0, 0);
        io<SO>::st(out + i, v);
    }
}

template <typename SI, typename SO>
__global__ void k_from_dev(const SI* __restrict__ in, SO* __restrict__ out, LatTab t, long long ncanon, int nrhs) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long V = t.off[t.nlat], n = 12 * V;
    if (i >= n * nrhs) return;
    const long long r = i / n, e = i - r * n;
    const int comp = (int)(e / V);
    const uint32_t s = (uint32_t)(e - comp * V);
    int k;
    uint32_t sl;
    if (!lat_site(t, s, k, sl)) return;
    SO* o = out + r * ncanon + 12LL * (t.coff[k] + sl) + comp;
    if constexpr (sizeof(SI) == 16 && sizeof(SO) == 16)
        *o = in[i];
    else
        *o = io<SI>::ld(in + i);
}

static inline dim3 grid_for(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

void to_device_layout(lqt_ctx* c, const double2* canon, double2* dev, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL((k_to_dev<double2, double2>), grid_for(n, 256), dim3(256), 0, c->stream, canon, dev, c->g.lat,
                       12LL * c->g.canon_sites, nrhs);
    LQT_HIP(hipGetLastError());
}
void from_device_layout(lqt_ctx* c, const double2* dev, double2* canon, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL((k_from_dev<double2, double2>), grid_for(n, 256), dim3(256), 0, c->stream, dev, canon,
                       c->g.lat, 12LL * c->g.canon_sites, nrhs);
    LQT_HIP(hipGetLastError());
}

template <typename S>
void convert_in_c64(lqt_ctx* c, const float2* canon, S* dev, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL((k_to_dev<float2, S>), grid_for(n, 256), dim3(256), 0, c->stream, canon, dev, c->g.lat,
                       12LL * c->g.canon_sites, nrhs);
    LQT_HIP(hipGetLastError());
}
template <typename S>
void convert_out_c64(lqt_ctx* c, const S* dev, float2* canon, int nrhs) {
    long long n = 12LL * c->g.V * nrhs;
    if (n == 0) return;
    hipLaunchKernelGGL((k_from_dev<S, float2>), grid_for(n, 256), dim3(256), 0, c->stream, dev, canon, c->g.lat,
                       12LL * c->g.canon_sites, nrhs);
    LQT_HIP(hipGetLastError());
}

template void convert_in_c64<float2>(lqt_ctx*, const float2*, float2*, int);
template void convert_in_c64<h2>(lqt_ctx*, const float2*, h2*, int);
template void convert_in_c64<b2>(lqt_ctx*, const float2*, b2*, int);
template void convert_out_c64<float2>(lqt_ctx*, const float2*, float2*, int);
template void convert_out_c64<h2>(lqt_ctx*, const h2*, float2*, int);
template void convert_out_c64<b2>(lqt_ctx*, const b2*, float2*, int);

}  // namespace lqt

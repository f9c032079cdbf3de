// Field-level BLAS on FP64 device-layout fields, and the Rademacher probes.
//
// Probes (Section 1: real +-1 entries, E[z_i z_j] = delta_ij): entry i (index
// 12*site + 3*spin + colour within its lattice) of probe j is 1 - 2*bit63(h(seed ^ h(j ^
// h(i)))) with h the SplitMix64 output function of Steele, Lea and Flood (OOPSLA 2014).  They
// are generated wherever they are consumed instead of being stored; every lattice of a
// multi-lattice context gets the probes a context of that lattice alone would, and padding
// sites get zeros.
#include "lqt_internal.h"
#include "blas.h"

namespace lqt {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double probe_entry(uint64_t seed, uint64_t j, uint64_t i) {
    return (sm64(seed ^ sm64(j ^ sm64(i))) >> 63) ? -1.0 : 1.0;
}

// partial |x_f|^2 per (block, field): grid (nsb, nf)
__global__ __launch_bounds__(256) void k_norm2_part(const double2* __restrict__ x, int V, double* __restrict__ part) {
    __shared__ double red[4];
    const int f = blockIdx.y, s = blockIdx.x * 256 + threadIdx.x;
    const long long n = 12LL * V;
    double a = 0;
    if (s < V)
#pragma unroll
        for (int c = 0; c < 12; c++) {
            double2 v = x[f * n + (long long)c * V + s];
            a += v.x * v.x + v.y * v.y;
        }
    a = wsum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)f * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_rows(const double* __restrict__ part, int nparts, double* __restrict__ out) {
    const int f = blockIdx.x;
    double a = 0;
    for (int k = threadIdx.x; k < nparts; k += 64) a += part[(long long)f * nparts + k];
    a = wsum(a);
    if (threadIdx.x == 0) out[f] = a;
}

void norm2_fields(lqt_ctx* c, const double2* x, int nf, double* out_dev) {
    if (nf <= 0) return;
    const int nsb = (c->g.V + 255) / 256;
    c->scratch[6].ensure(sizeof(double) * (size_t)nsb * nf);
    hipLaunchKernelGGL(k_norm2_part, dim3(nsb, nf), dim3(256), 0, c->stream, x, c->g.V, c->scratch[6].as<double>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_rows, dim3(nf), dim3(64), 0, c->stream, c->scratch[6].as<double>(), nsb, out_dev);
    LQT_HIP(hipGetLastError());
}

// out[j] = probe (seed, j0 + j) in device layout
__global__ __launch_bounds__(256) void k_probe_gen(uint64_t seed, long long j0, LatTab t, double2* __restrict__ out) {
    const int V = t.off[t.nlat];
    const int j = blockIdx.y, s = blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const long long n = 12LL * V;
    int k;
    uint32_t sl;
    const bool ok = lat_site(t, (uint32_t)s, k, sl);
#pragma unroll
    for (int c = 0; c < 12; c++)
        out[j * n + (long long)c * V + s] =
            make_double2(ok ? probe_entry(seed, (uint64_t)(j0 + j), (uint64_t)(12LL * sl + c)) : 0.0, 0.0);
}

void probes_gen(lqt_ctx* c, uint64_t seed, long long j0, int nprobes, double2* out) {
    if (nprobes <= 0) return;
    hipLaunchKernelGGL(k_probe_gen, dim3((c->g.V + 255) / 256, nprobes), dim3(256), 0, c->stream, seed, j0, c->g.lat,
                       out);
    LQT_HIP(hipGetLastError());
}

// Partition probes (the partition basis H of Algorithms 1 and 2: spin-colour dilution and
// hierarchical probing, Section 1).  Vector p = j q + m nd + cc (q = hp nd vectors per draw,
// nd = 12 with dilution, else 1) is the Rademacher probe j times the probing sign h_m of
// each site, restricted to spin-colour component cc when diluting.  h_m(x) is -1 to the sum
// over the set bits beta of m of f_beta(x), with the nested bit functions of level
// l = beta / 4 on the coordinate bits x_l = (x >> l) & 1:
//   f_{4l} = x_l + y_l + z_l + t_l (red-black at level l), f_{4l+1} = x_l, f_{4l+2} = y_l,
//   f_{4l+3} = z_l,
// so the first 2^{4i} signs span the indicators of the sites congruent modulo 2^i in every
// direction (the closing colours).
__device__ __forceinline__ int hp_parity(uint32_t m, int x, int y, int z, int t) {
    int par = 0;
    for (int beta = 0; (m >> beta) != 0u; beta++) {
        if (!((m >> beta) & 1u)) continue;
        const int l = beta >> 2;
        const int xl = (x >> l) & 1, yl = (y >> l) & 1, zl = (z >> l) & 1, tl = (t >> l) & 1;
        const int w = beta & 3;
        par += w == 0 ? xl + yl + zl + tl : (w == 1 ? xl : (w == 2 ? yl : zl));
    }
    return par & 1;
}

__global__ __launch_bounds__(256) void k_partition_probe_gen(uint64_t seed, long long p0, int hp, int nd, int L0,
                                                             int L1, int L2, int V, double2* __restrict__ out) {
    const int f = blockIdx.y, s = blockIdx.x * 256 + threadIdx.x;
    if (s >= V) return;
    const long long p = p0 + f;
    const int q = hp * nd;
    const long long j = p / q;
    const int r = (int)(p % q), m = r / nd, cc = r % nd;
    const int x = s % L0, y = (s / L0) % L1, z = (s / (L0 * L1)) % L2, t = s / (L0 * L1 * L2);
    const double sg = hp_parity((uint32_t)m, x, y, z, t) ? -1.0 : 1.0;
    const long long n = 12LL * V;
#pragma unroll
    for (int c = 0; c < 12; c++)
        out[f * n + (long long)c * V + s] =
            make_double2((nd == 1 || c == cc) ? sg * probe_entry(seed, (uint64_t)j, (uint64_t)(12LL * s + c)) : 0.0, 0.0);
}

void check_partition(const lqt_ctx* c, int hp_vectors, int dilute) {
    LQT_CHECK(c->g.lat.nlat == 1, LQT_EINVAL, "partition probes serve single-lattice contexts");
    LQT_CHECK(dilute == 0 || dilute == 1, LQT_EINVAL, "dilute must be 0 or 1");
    LQT_CHECK(hp_vectors >= 1 && hp_vectors <= (1 << 20) && !(hp_vectors & (hp_vectors - 1)), LQT_EINVAL,
              "hp_vectors must be a power of two (1 = no probing)");
    // the highest level l of the nested colourings needs extents divisible by 2^(l+1)
    int b = 0;
    while ((1 << b) < hp_vectors) b++;
    if (b > 0) {
        const int m = 2 << ((b - 1) / 4);
        for (int d = 0; d < 4; d++)
            LQT_CHECK(c->g.L[d] % m == 0, LQT_EINVAL,
                      std::to_string(hp_vectors) + " probing vectors need extents divisible by " + std::to_string(m));
    }
}

void partition_probes_gen(lqt_ctx* c, uint64_t seed, long long p0, int nvec, int hp, int dilute, double2* out) {
    if (nvec <= 0) return;
    LQT_CHECK(nvec <= 65535, LQT_EINVAL, "partition probes: at most 65535 vectors per launch");
    hipLaunchKernelGGL(k_partition_probe_gen, dim3((c->g.V + 255) / 256, nvec), dim3(256), 0, c->stream, seed, p0, hp,
                       dilute ? 12 : 1, c->g.L[0], c->g.L[1], c->g.L[2], c->g.V, out);
    LQT_HIP(hipGetLastError());
}

// partial sums of z_j^T y_j (complex) per (block, probe): y device layout FP64
__global__ __launch_bounds__(256) void k_probe_dot_part(uint64_t seed, long long j0, const double2* __restrict__ y,
                                                        LatTab t, double2* __restrict__ part) {
    __shared__ double red[4][2];
    const int V = t.off[t.nlat];
    const int j = blockIdx.y, s = blockIdx.x * 256 + threadIdx.x;
    const long long n = 12LL * V;
    double a = 0, b = 0;
    int k;
    uint32_t sl;
    if (s < V && lat_site(t, (uint32_t)s, k, sl))
#pragma unroll
        for (int c = 0; c < 12; c++) {
            double z = probe_entry(seed, (uint64_t)(j0 + j), (uint64_t)(12LL * sl + c));
            double2 v = y[j * n + (long long)c * V + s];
            a += z * v.x;
            b += z * v.y;
        }
    a = wsum(a);
    b = wsum(b);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        part[(long long)j * gridDim.x + blockIdx.x] =
            make_double2(red[0][0] + red[1][0] + red[2][0] + red[3][0], red[0][1] + red[1][1] + red[2][1] + red[3][1]);
}

__global__ void k_sum_rows2(const double2* __restrict__ part, int nparts, double2* __restrict__ out) {
    const int f = blockIdx.x;
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < nparts; k += 64) {
        double2 p = part[(long long)f * nparts + k];
        a += p.x;
        b += p.y;
    }
    a = wsum(a);
    b = wsum(b);
    if (threadIdx.x == 0) out[f] = make_double2(a, b);
}

// out[f * nlat + k] = sum of the block partials of row f over the blocks of lattice k
// (256-site blocks; lattices start on block boundaries)
template <typename T>
__global__ void k_sum_rows_lat(const T* __restrict__ part, int nparts, LatTab t, T* __restrict__ out) {
    const int f = blockIdx.x, k = blockIdx.y;
    const int b0 = t.off[k] / 256, b1 = (t.off[k + 1] + 255) / 256;
    double a = 0, b = 0;
    for (int q = b0 + threadIdx.x; q < b1 && q < nparts; q += 64) {
        if constexpr (sizeof(T) == 16) {
            const double2 p = part[(long long)f * nparts + q];
            a += p.x;
            b += p.y;
        } else {
            a += part[(long long)f * nparts + q];
        }
    }
    a = wsum(a);
    b = wsum(b);
    if (threadIdx.x == 0) {
        if constexpr (sizeof(T) == 16)
            out[f * t.nlat + k] = make_double2(a, b);
        else
            out[f * t.nlat + k] = a;
    }
}

void probe_dots(lqt_ctx* c, uint64_t seed, long long j0, const double2* y, int nprobes, double2* out_dev,
                bool per_lattice) {
    if (nprobes <= 0) return;
    const int nsb = (c->g.V + 255) / 256;
    c->scratch[6].ensure(sizeof(double2) * (size_t)nsb * nprobes);
    hipLaunchKernelGGL(k_probe_dot_part, dim3(nsb, nprobes), dim3(256), 0, c->stream, seed, j0, y, c->g.lat,
                       c->scratch[6].as<double2>());
    LQT_HIP(hipGetLastError());
    if (per_lattice)
        hipLaunchKernelGGL(k_sum_rows_lat<double2>, dim3(nprobes, c->g.lat.nlat), dim3(64), 0, c->stream,
                           c->scratch[6].as<double2>(), nsb, c->g.lat, out_dev);
    else
        hipLaunchKernelGGL(k_sum_rows2, dim3(nprobes), dim3(64), 0, c->stream, c->scratch[6].as<double2>(), nsb,
                           out_dev);
    LQT_HIP(hipGetLastError());
}

void sum_partials_lattices(lqt_ctx* c, const double* part, int nparts, int nf, double* out_dev) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(k_sum_rows_lat<double>, dim3(nf, c->g.lat.nlat), dim3(64), 0, c->stream, part, nparts,
                       c->g.lat, out_dev);
    LQT_HIP(hipGetLastError());
}

void norm2_lattices(lqt_ctx* c, const double2* x, int nf, double* out_dev) {
    if (nf <= 0) return;
    const int nsb = (c->g.V + 255) / 256;
    c->scratch[6].ensure(sizeof(double) * (size_t)nsb * nf);
    hipLaunchKernelGGL(k_norm2_part, dim3(nsb, nf), dim3(256), 0, c->stream, x, c->g.V, c->scratch[6].as<double>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_rows_lat<double>, dim3(nf, c->g.lat.nlat), dim3(64), 0, c->stream,
                       c->scratch[6].as<double>(), nsb, c->g.lat, out_dev);
    LQT_HIP(hipGetLastError());
}

// partial conj(x_f)^T y_f per (block, field)
__global__ __launch_bounds__(256) void k_dot_part(const double2* __restrict__ x, const double2* __restrict__ y, int V,
                                                  double2* __restrict__ part) {
    __shared__ double red[4][2];
    const int f = blockIdx.y, s = blockIdx.x * 256 + threadIdx.x;
    const long long n = 12LL * V;
    double a = 0, b = 0;
    if (s < V)
#pragma unroll
        for (int c = 0; c < 12; c++) {
            double2 u = x[f * n + (long long)c * V + s], v = y[f * n + (long long)c * V + s];
            a += u.x * v.x + u.y * v.y;
            b += u.x * v.y - u.y * v.x;
        }
    a = wsum(a);
    b = wsum(b);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        part[(long long)f * gridDim.x + blockIdx.x] =
            make_double2(red[0][0] + red[1][0] + red[2][0] + red[3][0], red[0][1] + red[1][1] + red[2][1] + red[3][1]);
}

void dot_fields(lqt_ctx* c, const double2* x, const double2* y, int nf, double2* out_dev) {
    if (nf <= 0) return;
    const int nsb = (c->g.V + 255) / 256;
    c->scratch[6].ensure(sizeof(double2) * (size_t)nsb * nf);
    hipLaunchKernelGGL(k_dot_part, dim3(nsb, nf), dim3(256), 0, c->stream, x, y, c->g.V, c->scratch[6].as<double2>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_rows2, dim3(nf), dim3(64), 0, c->stream, c->scratch[6].as<double2>(), nsb, out_dev);
    LQT_HIP(hipGetLastError());
}

// x <- g5 x (flip spins 2, 3) for nf FP64 fields
__global__ void k_g5(double2* __restrict__ x, int V, long long total) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    long long n = 12LL * V;
    long long e = i % n;
    int comp = (int)(e / V);
    if (comp >= 6) {
        double2 v = x[i];
        x[i] = make_double2(-v.x, -v.y);
    }
}

void gamma5_fields(lqt_ctx* c, double2* x, int nf) {
    long long total = 12LL * c->g.V * nf;
    if (total == 0) return;
    hipLaunchKernelGGL(k_g5, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, x, c->g.V, total);
    LQT_HIP(hipGetLastError());
}

// NaN / Inf scan of n doubles: bad[0] = 1 if any is not finite (flag must be zeroed first)
__global__ void k_nan(const double* __restrict__ p, size_t n, int* __restrict__ bad) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    int b = 0;
    for (; i < n; i += st) {
        double v = p[i];
        if (!(v - v == 0.0)) b = 1;
    }
    if (b) bad[0] = 1;
}

bool has_nonfinite(lqt_ctx* c, const double* p, size_t n) {
    c->scratch[5].ensure(sizeof(int));
    int* d = c->scratch[5].as<int>();
    LQT_HIP(hipMemsetAsync(d, 0, sizeof(int), c->stream));
    if (n) {
        hipLaunchKernelGGL(k_nan, dim3(1024), dim3(256), 0, c->stream, p, n, d);
        LQT_HIP(hipGetLastError());
    }
    int h = 0;
    LQT_HIP(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    LQT_HIP(hipStreamSynchronize(c->stream));
    return h != 0;
}

}  // namespace lqt

namespace lqt {

// Complex Gaussian fields (unit variance per real part) from a counter hash and Box-Muller:
// entry (f, i) uses h(seed ^ h(f ^ h(2i))) and h(seed ^ h(f ^ h(2i+1))) as uniforms.
__global__ void k_gauss(uint64_t seed, long long n, int nf, double2* __restrict__ out) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nf) return;
    long long f = e / n, i = e - f * n;
    uint64_t h1 = sm64(seed ^ sm64((uint64_t)f ^ sm64((uint64_t)(2 * i))));
    uint64_t h2 = sm64(seed ^ sm64((uint64_t)f ^ sm64((uint64_t)(2 * i + 1))));
    double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
    double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    double r = sqrt(-2.0 * log(u1));
    out[e] = make_double2(r * cos(6.283185307179586 * u2), r * sin(6.283185307179586 * u2));
}

void gaussian_fields(lqt_ctx* c, uint64_t seed, long long n, int nf, double2* out) {
    long long tot = n * nf;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_gauss, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, seed, n, nf, out);
    LQT_HIP(hipGetLastError());
}

// partial |w_f - theta_f q_f|^2 over generic vectors of length n (grid: chunks x fields)
__global__ __launch_bounds__(256) void k_eigres_part(const double2* __restrict__ W, const double2* __restrict__ Q,
                                                     const double* __restrict__ theta, long long n,
                                                     double* __restrict__ part) {
    __shared__ double red[4];
    const int f = blockIdx.y;
    const double th = theta[f];
    double a = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double2 w = W[f * n + i], q = Q[f * n + i];
        double x = w.x - th * q.x, y = w.y - th * q.y;
        a += x * x + y * y;
    }
    a = wsum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)f * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

void eig_residual_norms(lqt_ctx* c, const double2* W, const double2* Q, const double* theta_dev, long long n, int nf,
                        double* out_dev) {
    if (nf <= 0) return;
    const int nb = 256;
    c->scratch[6].ensure(sizeof(double) * (size_t)nb * nf);
    hipLaunchKernelGGL(k_eigres_part, dim3(nb, nf), dim3(256), 0, c->stream, W, Q, theta_dev, n,
                       c->scratch[6].as<double>());
    LQT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_rows, dim3(nf), dim3(64), 0, c->stream, c->scratch[6].as<double>(), nb, out_dev);
    LQT_HIP(hipGetLastError());
}

}  // namespace lqt

/*
 * Plain FP64 CPU oracle for the deflated Hutchinson trace estimator of the
 * Wilson-Dirac operator (Romero, Stathopoulos, Orginos, "Multigrid deflation for
 * Lattice QCD", arXiv:1909.12234).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or load
 * this file.  It is deliberately slow and literal: complex double everywhere, natural
 * site order, the full 4x4 (spin) times 3x3 (colour) form of every hopping term with
 * no spin projection, and textbook restarted GMRES with modified Gram-Schmidt.  It
 * shares no code, table or header with the HIP path.
 *
 * Geometry: dims = (Lx, Ly, Lz, Lt), site s = x + Lx*(y + Ly*(z + Lz*t)); spinor
 * component 12*s + 3*spin + colour; links U[((s*4 + mu)*3 + a)*3 + b], mu = 0..3 for
 * x, y, z, t.  Periodic in every direction, with an extra factor -1 on hops that cross
 * the time boundary when `antiperiodic` is set.
 *
 * Operator (the Wilson-Dirac matrix whose trace of the inverse the paper estimates):
 *   (A psi)(x) = (4+m) psi(x)
 *              - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * with DeGrand-Rossi gamma matrices (g5 = g1 g2 g3 g4 = diag(1,1,-1,-1)).
 * A^+ is formed from the definition of the adjoint (the two projectors swap), not from
 * g5-hermiticity, so the tests can check g5 A g5 = A^+ as an independent fact.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { ORC_A = 0, ORC_ADAG = 1, ORC_AG5 = 2, ORC_G5A = 3 };

/* ---------------------------------------------------------------- gamma matrices */
/* DeGrand-Rossi basis, written out entry by entry. */
static void gamma_matrix(int mu, cplx g[4][4]) {
    memset(g, 0, sizeof(cplx) * 16);
    const cplx Im = _Complex_I;
    switch (mu) {
    case 0: /* gamma_1 */
        g[0][3] = Im; g[1][2] = Im; g[2][1] = -Im; g[3][0] = -Im; break;
    case 1: /* gamma_2 */
        g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1; break;
    case 2: /* gamma_3 */
        g[0][2] = Im; g[1][3] = -Im; g[2][0] = -Im; g[3][1] = Im; break;
    default: /* gamma_4 */
        g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1; break;
    }
}

/* Exported so the tests can check the Clifford algebra of the oracle's own table. */
void orc_gamma(int mu, double *out /* 4x4 complex, interleaved re/im */) {
    cplx g[4][4];
    gamma_matrix(mu, g);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            out[2 * (4 * i + j)] = creal(g[i][j]);
            out[2 * (4 * i + j) + 1] = cimag(g[i][j]);
        }
}

/* ---------------------------------------------------------------- geometry */
typedef struct {
    int L[4];
    long V;
} geom_t;

static geom_t make_geom(const int *dims) {
    geom_t g;
    for (int i = 0; i < 4; i++) g.L[i] = dims[i];
    g.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return g;
}

static void site_coords(const geom_t *g, long s, int c[4]) {
    for (int i = 0; i < 4; i++) {
        c[i] = (int)(s % g->L[i]);
        s /= g->L[i];
    }
}

static long coords_site(const geom_t *g, const int c[4]) {
    return c[0] + (long)g->L[0] * (c[1] + (long)g->L[1] * (c[2] + (long)g->L[2] * c[3]));
}

/* neighbour of site s one step in direction mu (dir = +1 or -1); *crossed_t is set
 * when the hop wraps around the time boundary. */
static long neighbour(const geom_t *g, long s, int mu, int dir, int *crossed_t) {
    int c[4];
    site_coords(g, s, c);
    int v = c[mu] + dir;
    *crossed_t = 0;
    if (v < 0) { v += g->L[mu]; if (mu == 3) *crossed_t = 1; }
    if (v >= g->L[mu]) { v -= g->L[mu]; if (mu == 3) *crossed_t = 1; }
    c[mu] = v;
    return coords_site(g, c);
}

/* ---------------------------------------------------------------- operator */
static void apply_wilson_one(const geom_t *g, double mass, int antiperiodic, const cplx *U,
                             int dagger, const cplx *in, cplx *out) {
    cplx gam[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, gam[mu]);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; s++) {
        cplx acc[4][3];
        for (int sp = 0; sp < 4; sp++)
            for (int c = 0; c < 3; c++) acc[sp][c] = (4.0 + mass) * in[12 * s + 3 * sp + c];
        for (int mu = 0; mu < 4; mu++) {
            /* projector signs: A uses (1 - g) forward and (1 + g) backward, A^+ swaps them */
            double fsign = dagger ? +1.0 : -1.0; /* forward projector 1 + fsign*g */
            double bsign = -fsign;
            int crossed;
            /* forward hop: U_mu(x) psi(x+mu) */
            long sf = neighbour(g, s, mu, +1, &crossed);
            double bc = (antiperiodic && crossed) ? -1.0 : 1.0;
            const cplx *Uf = U + (s * 4 + mu) * 9;
            cplx chi[4][3];
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int b = 0; b < 3; b++) t += Uf[3 * a + b] * in[12 * sf + 3 * sp + b];
                    chi[sp][a] = t;
                }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int q = 0; q < 4; q++) {
                        cplx proj = (sp == q ? 1.0 : 0.0) + fsign * gam[mu][sp][q];
                        t += proj * chi[q][a];
                    }
                    acc[sp][a] -= 0.5 * bc * t;
                }
            /* backward hop: U_mu(x-mu)^+ psi(x-mu) */
            long sb = neighbour(g, s, mu, -1, &crossed);
            bc = (antiperiodic && crossed) ? -1.0 : 1.0;
            const cplx *Ub = U + (sb * 4 + mu) * 9;
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int b = 0; b < 3; b++) t += conj(Ub[3 * b + a]) * in[12 * sb + 3 * sp + b];
                    chi[sp][a] = t;
                }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int q = 0; q < 4; q++) {
                        cplx proj = (sp == q ? 1.0 : 0.0) + bsign * gam[mu][sp][q];
                        t += proj * chi[q][a];
                    }
                    acc[sp][a] -= 0.5 * bc * t;
                }
        }
        for (int sp = 0; sp < 4; sp++)
            for (int c = 0; c < 3; c++) out[12 * s + 3 * sp + c] = acc[sp][c];
    }
}

static void gamma5_inplace(long V, cplx *v) {
    for (long s = 0; s < V; s++)
        for (int sp = 2; sp < 4; sp++)
            for (int c = 0; c < 3; c++) v[12 * s + 3 * sp + c] = -v[12 * s + 3 * sp + c];
}

static void apply_op(const geom_t *g, double mass, int antiperiodic, const cplx *U, int op,
                     const cplx *in, cplx *out, cplx *tmp) {
    long N = 12 * g->V;
    switch (op) {
    case ORC_A: apply_wilson_one(g, mass, antiperiodic, U, 0, in, out); break;
    case ORC_ADAG: apply_wilson_one(g, mass, antiperiodic, U, 1, in, out); break;
    case ORC_AG5:
        memcpy(tmp, in, sizeof(cplx) * N);
        gamma5_inplace(g->V, tmp);
        apply_wilson_one(g, mass, antiperiodic, U, 0, tmp, out);
        break;
    default:
        apply_wilson_one(g, mass, antiperiodic, U, 0, in, out);
        gamma5_inplace(g->V, out);
        break;
    }
}

/* out[r] = op(in[r]) for r < nrhs; in/out are nrhs consecutive spinor fields. */
int orc_apply(const int *dims, double mass, int antiperiodic, const double *links, int op,
              const double *in, double *out, int nrhs) {
    geom_t g = make_geom(dims);
    long N = 12 * g.V;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * N);
    if (!tmp) return -1;
    for (int r = 0; r < nrhs; r++)
        apply_op(&g, mass, antiperiodic, (const cplx *)links, op, (const cplx *)in + r * N,
                 (cplx *)out + r * N, tmp);
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------- GMRES(m) */
static double vnorm(long n, const cplx *v) {
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return sqrt(s);
}

static cplx vdot(long n, const cplx *a, const cplx *b) { /* a^H b */
    cplx s = 0;
    for (long i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

/*
 * Restarted GMRES(m) for op(x) = b, x0 = 0, modified Gram-Schmidt Arnoldi, Givens
 * rotations on the Hessenberg matrix.  A cycle ends after m steps or when the Arnoldi
 * residual estimate falls below xi*||b||; every restart recomputes the true residual
 * b - op(x), and the solve stops only when that true residual is <= xi*||b|| (the
 * stopping rule of an inexact solve A^{-1}_xi, Section 1) or maxit steps have run.
 * Returns 0 when converged, 1 otherwise.  iters = Arnoldi steps, relres = true
 * residual / ||b|| at exit.
 */
int orc_gmres(const int *dims, double mass, int antiperiodic, const double *links, int op,
              const double *b_, double *x_, int m, double xi, int maxit, int *iters,
              double *relres) {
    geom_t g = make_geom(dims);
    long N = 12 * g.V;
    const cplx *U = (const cplx *)links;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *Vb = (cplx *)malloc(sizeof(cplx) * N * (m + 1));
    cplx *w = (cplx *)malloc(sizeof(cplx) * N);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * N);
    cplx *H = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx)); /* H[i*m + j] */
    double *sn_r = (double *)malloc(sizeof(double) * m); /* rotations: [c s; -conj(s) c]: c real */
    cplx *sn = (cplx *)malloc(sizeof(cplx) * m);
    cplx *gvec = (cplx *)malloc(sizeof(cplx) * (m + 1));
    cplx *y = (cplx *)malloc(sizeof(cplx) * m);
    if (!Vb || !w || !tmp || !H || !sn_r || !sn || !gvec || !y) return -1;
    memset(x, 0, sizeof(cplx) * N);
    double bnorm = vnorm(N, b);
    double target = xi * bnorm;
    int its = 0, status = 1;
    double rel = 1.0;
    if (bnorm == 0.0) { status = 0; rel = 0.0; goto done; }
    for (;;) {
        /* true residual r = b - op(x) */
        apply_op(&g, mass, antiperiodic, U, op, x, w, tmp);
        for (long i = 0; i < N; i++) w[i] = b[i] - w[i];
        double beta = vnorm(N, w);
        rel = beta / bnorm;
        if (beta <= target) { status = 0; break; }
        if (its >= maxit) break;
        for (long i = 0; i < N; i++) Vb[i] = w[i] / beta;
        memset(gvec, 0, sizeof(cplx) * (m + 1));
        gvec[0] = beta;
        int j;
        int kdim = 0;
        for (j = 0; j < m && its < maxit; j++) {
            cplx *vj = Vb + (long)j * N;
            cplx *vn = Vb + (long)(j + 1) * N;
            apply_op(&g, mass, antiperiodic, U, op, vj, vn, tmp);
            its++;
            for (int i = 0; i <= j; i++) { /* modified Gram-Schmidt */
                cplx h = vdot(N, Vb + (long)i * N, vn);
                H[i * m + j] = h;
                const cplx *vi = Vb + (long)i * N;
                for (long k = 0; k < N; k++) vn[k] -= h * vi[k];
            }
            double hn = vnorm(N, vn);
            H[(j + 1) * m + j] = hn;
            if (hn > 0)
                for (long k = 0; k < N; k++) vn[k] /= hn;
            /* apply previous rotations to column j */
            for (int i = 0; i < j; i++) {
                cplx h0 = H[i * m + j], h1 = H[(i + 1) * m + j];
                H[i * m + j] = sn_r[i] * h0 + sn[i] * h1;
                H[(i + 1) * m + j] = -conj(sn[i]) * h0 + sn_r[i] * h1;
            }
            /* new rotation zeroing H[j+1][j] */
            cplx a = H[j * m + j];
            double bb = creal(H[(j + 1) * m + j]);
            double r = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + bb * bb);
            double c;
            cplx s;
            if (r == 0) { c = 1; s = 0; }
            else if (cabs(a) == 0) { c = 0; s = 1; r = bb; }
            else {
                double absa = cabs(a);
                c = absa / r;
                s = (a / absa) * bb / r; /* then -conj(s)*a + c*bb = 0 */
            }
            sn_r[j] = c;
            sn[j] = s;
            H[j * m + j] = c * a + s * bb;
            H[(j + 1) * m + j] = 0;
            cplx g0 = gvec[j];
            gvec[j] = c * g0;
            gvec[j + 1] = -conj(s) * g0;
            kdim = j + 1;
            if (cabs(gvec[j + 1]) <= target || hn == 0) { j++; break; }
        }
        /* back substitution H y = g, x += V y */
        for (int i = kdim - 1; i >= 0; i--) {
            cplx t = gvec[i];
            for (int k = i + 1; k < kdim; k++) t -= H[i * m + k] * y[k];
            y[i] = t / H[i * m + i];
        }
        for (int i = 0; i < kdim; i++) {
            const cplx *vi = Vb + (long)i * N;
            for (long k = 0; k < N; k++) x[k] += y[i] * vi[k];
        }
    }
done:
    if (iters) *iters = its;
    if (relres) *relres = rel;
    free(Vb); free(w); free(tmp); free(H); free(sn_r); free(sn); free(gvec); free(y);
    return status;
}

/* ---------------------------------------------------------------- probes */
/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the first output of the generator
 * whose state is x, used as a 64-bit mixing hash. */
uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Rademacher probe entries z_{j,i} = 1 - 2*bit63(h(seed ^ h(j ^ h(i)))), i = 0..N-1
 * (global spin-colour-site index), j = j0 .. j0+nprobes-1; real, so only +-1 is stored. */
void orc_probes(uint64_t seed, long j0, int nprobes, long N, double *out) {
    for (int jj = 0; jj < nprobes; jj++) {
        uint64_t j = (uint64_t)(j0 + jj);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) {
            uint64_t h = orc_splitmix64(seed ^ orc_splitmix64(j ^ orc_splitmix64((uint64_t)i)));
            out[(long)jj * N + i] = (h >> 63) ? -1.0 : 1.0;
        }
    }
}

/* ---------------------------------------------------------------- transport net */
/*
 * Forward pass of a linear gauge-equivariant parallel-transport network.  A field with
 * F features holds F colour 3-vectors per site, stored [site][feature][colour].  One
 * layer maps F_in -> F_out features:
 *   out_f(x) = sum_{p} sum_g W[p][f][g] * (T_p v_g)(x)
 * over the nine paths p = 0 (identity), 1+2mu (+mu), 2+2mu (-mu), where
 *   (T_{+mu} v)(x) = U_mu(x) v(x+mu),   (T_{-mu} v)(x) = U_mu(x-mu)^+ v(x-mu)
 * and hops across the time boundary pick up the same -1 as the fermion operator.
 * feats[0..nlayers] are the feature counts; weights are concatenated per layer,
 * W_l[p][f][g] complex (9 * F_out * F_in entries).
 */
static void transport(const geom_t *g, int antiperiodic, const cplx *U, int p, int F,
                      const cplx *in, cplx *out) {
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; s++) {
        if (p == 0) {
            for (int f = 0; f < F; f++)
                for (int a = 0; a < 3; a++) out[(s * F + f) * 3 + a] = in[(s * F + f) * 3 + a];
            continue;
        }
        int mu = (p - 1) / 2, fwd = ((p - 1) % 2) == 0;
        int crossed;
        long sn = neighbour(g, s, mu, fwd ? +1 : -1, &crossed);
        double bc = (antiperiodic && crossed) ? -1.0 : 1.0;
        const cplx *L = fwd ? U + (s * 4 + mu) * 9 : U + (sn * 4 + mu) * 9;
        for (int f = 0; f < F; f++)
            for (int a = 0; a < 3; a++) {
                cplx t = 0;
                for (int b = 0; b < 3; b++) {
                    cplx l = fwd ? L[3 * a + b] : conj(L[3 * b + a]);
                    t += l * in[(sn * F + f) * 3 + b];
                }
                out[(s * F + f) * 3 + a] = bc * t;
            }
    }
}

int orc_ptc_forward(const int *dims, int antiperiodic, const double *links, int nlayers,
                    const int *feats, const double *weights, const double *in, double *out) {
    geom_t g = make_geom(dims);
    const cplx *U = (const cplx *)links;
    const cplx *W = (const cplx *)weights;
    int fmax = 0;
    for (int l = 0; l <= nlayers; l++) fmax = feats[l] > fmax ? feats[l] : fmax;
    cplx *cur = (cplx *)malloc(sizeof(cplx) * g.V * fmax * 3);
    cplx *nxt = (cplx *)malloc(sizeof(cplx) * g.V * fmax * 3);
    cplx *tp = (cplx *)malloc(sizeof(cplx) * g.V * fmax * 3);
    if (!cur || !nxt || !tp) return -1;
    memcpy(cur, in, sizeof(cplx) * g.V * feats[0] * 3);
    for (int l = 0; l < nlayers; l++) {
        int Fi = feats[l], Fo = feats[l + 1];
        memset(nxt, 0, sizeof(cplx) * g.V * Fo * 3);
        for (int p = 0; p < 9; p++) {
            transport(&g, antiperiodic, U, p, Fi, cur, tp);
            const cplx *Wp = W + (long)p * Fo * Fi;
            for (long s = 0; s < g.V; s++)
                for (int f = 0; f < Fo; f++)
                    for (int a = 0; a < 3; a++) {
                        cplx t = 0;
                        for (int q = 0; q < Fi; q++) t += Wp[f * Fi + q] * tp[(s * Fi + q) * 3 + a];
                        nxt[(s * Fo + f) * 3 + a] += t;
                    }
        }
        W += 9L * Fo * Fi;
        cplx *sw = cur; cur = nxt; nxt = sw;
    }
    memcpy(out, cur, sizeof(cplx) * g.V * feats[nlayers] * 3);
    free(cur); free(nxt); free(tp);
    return 0;
}

/*
 * Plain FP64 Wilson-Dirac stencil and BiCGStab (oracle, test infrastructure only).
 *
 * Independent of the GPU library: no shared headers, helpers or layouts.
 * Written for obvious correctness: explicit 4x4 complex spin matrices, the
 * canonical lexicographic layout, one OpenMP loop over sites.
 *
 * Operator (plain Wilson, r = 1; the paper's Section 1 describes the Dirac
 * matrix only as a 4D nearest-neighbour operator with 4 spin x 3 colour
 * degrees of freedom per site):
 *   D psi(x) = (4+m) psi(x) - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                        + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
 * with -1 on hops across the t boundary when antiperiodic.  Chiral basis:
 * g_k = [[0, -i s_k], [i s_k, 0]], g_t = [[0, 1], [1, 0]].
 *
 * Layouts: spinor [t][z][y][x][spin 4][colour 3] complex128 (interleaved
 * re, im doubles); links [4][t][z][y][x][3][3] complex128.
 *
 * The linear solver (Algorithm 1 "Solve Ay = z", solver unspecified in the
 * paper) is textbook BiCGStab (van der Vorst 1992) on one right-hand side,
 * x0 = 0, stopped on the recurrence residual and confirmed on the true one.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static cplx G[4][4][4];   /* G[mu][row][col] */
static int g_init = 0;

static void init_gamma(void) {
    if (g_init) return;
    memset(G, 0, sizeof(G));
    /* Pauli matrices */
    cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                G[k][a][2 + b] = -I * s[k][a][b];
                G[k][2 + a][b] = I * s[k][a][b];
            }
    G[3][0][2] = 1; G[3][1][3] = 1; G[3][2][0] = 1; G[3][3][1] = 1;
    g_init = 1;
}

static long site_of(const int *L, int x, int y, int z, int t) {
    return (long)x + (long)L[0] * ((long)y + (long)L[1] * ((long)z + (long)L[2] * (long)t));
}

void o2_dslash(const int *L, double mass, int antiperiodic, const double *Ud,
               const double *ind, double *outd) {
    init_gamma();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    long V = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        int c[4];
        long r = n;
        c[0] = (int)(r % L[0]); r /= L[0];
        c[1] = (int)(r % L[1]); r /= L[1];
        c[2] = (int)(r % L[2]); r /= L[2];
        c[3] = (int)r;
        cplx acc[4][3];
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) acc[s][a] = (4.0 + mass) * in[12 * n + 3 * s + a];
        for (int mu = 0; mu < 4; mu++) {
            int cf[4] = {c[0], c[1], c[2], c[3]};
            int cb[4] = {c[0], c[1], c[2], c[3]};
            cf[mu] = (c[mu] + 1) % L[mu];
            cb[mu] = (c[mu] + L[mu] - 1) % L[mu];
            long nf = site_of(L, cf[0], cf[1], cf[2], cf[3]);
            long nb = site_of(L, cb[0], cb[1], cb[2], cb[3]);
            double phf = (antiperiodic && mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
            double phb = (antiperiodic && mu == 3 && c[3] == 0) ? -1.0 : 1.0;
            const cplx *Uf = U + 9 * ((long)mu * V + n);    /* U_mu(x)      */
            const cplx *Ub = U + 9 * ((long)mu * V + nb);   /* U_mu(x - mu) */
            /* colour multiply first: uf[s][a] = sum_b U(x)[a][b] psi(x+mu)[s][b],
               ub[s][a] = sum_b conj(U(x-mu)[b][a]) psi(x-mu)[s][b] */
            cplx uf[4][3], ub[4][3];
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++) {
                    cplx f = 0, b2 = 0;
                    for (int b = 0; b < 3; b++) {
                        f += Uf[3 * a + b] * in[12 * nf + 3 * s + b];
                        b2 += conj(Ub[3 * b + a]) * in[12 * nb + 3 * s + b];
                    }
                    uf[s][a] = f;
                    ub[s][a] = b2;
                }
            /* spin multiply: (1 - g_mu) and (1 + g_mu) */
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++) {
                    cplx f = 0, b2 = 0;
                    for (int t2 = 0; t2 < 4; t2++) {
                        cplx id = (s == t2) ? 1.0 : 0.0;
                        f += (id - G[mu][s][t2]) * uf[t2][a];
                        b2 += (id + G[mu][s][t2]) * ub[t2][a];
                    }
                    acc[s][a] += -0.5 * (phf * f + phb * b2);
                }
        }
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) out[12 * n + 3 * s + a] = acc[s][a];
    }
}

static cplx dotc(const cplx *a, const cplx *b, long n) {   /* a^H b */
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx p = conj(a[i]) * b[i];
        re += creal(p);
        im += cimag(p);
    }
    return re + I * im;
}

static double norm2(const cplx *a, long n) { return creal(dotc(a, a, n)); }

/* BiCGStab for D x = b (x starts at 0).  Returns 0 on convergence, 1 if maxiter
 * was reached, 2 on breakdown.  iters_out: iterations done; relres_out: true
 * relative residual ||b - D x|| / ||b|| at exit. */
int o2_bicgstab(const int *L, double mass, int antiperiodic, const double *Ud,
                const double *bd, double *xd, double tol, int maxiter,
                int *iters_out, double *relres_out) {
    long N = 12L * L[0] * L[1] * L[2] * L[3];
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = malloc(sizeof(cplx) * N), *rh = malloc(sizeof(cplx) * N);
    cplx *p = malloc(sizeof(cplx) * N), *v = malloc(sizeof(cplx) * N);
    cplx *s = malloc(sizeof(cplx) * N), *t = malloc(sizeof(cplx) * N);
    int status = 1, it = 0;
    for (long i = 0; i < N; i++) { x[i] = 0; r[i] = b[i]; rh[i] = b[i]; p[i] = 0; v[i] = 0; }
    double bn = sqrt(norm2(b, N));
    cplx rho = 1, alpha = 1, omega = 1;
    if (bn == 0.0) { status = 0; goto done; }
    for (it = 0; it < maxiter;) {
        cplx rho_new = dotc(rh, r, N);
        if (cabs(rho_new) == 0.0 || cabs(omega) == 0.0) { status = 2; break; }
        cplx beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        o2_dslash(L, mass, antiperiodic, Ud, (const double *)p, (double *)v);
        cplx rv = dotc(rh, v, N);
        if (cabs(rv) == 0.0) { status = 2; break; }
        alpha = rho / rv;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
        o2_dslash(L, mass, antiperiodic, Ud, (const double *)s, (double *)t);
        double tt = norm2(t, N);
        omega = (tt == 0.0) ? 0.0 : dotc(t, s, N) / tt;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        it++;
        if (sqrt(norm2(r, N)) <= tol * bn) {
            /* confirm on the true residual */
            o2_dslash(L, mass, antiperiodic, Ud, (const double *)x, (double *)t);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < N; i++) r[i] = b[i] - t[i];
            if (sqrt(norm2(r, N)) <= tol * bn) { status = 0; break; }
        }
    }
done:
    o2_dslash(L, mass, antiperiodic, Ud, (const double *)x, (double *)t);
    for (long i = 0; i < N; i++) s[i] = b[i] - t[i];
    *relres_out = (bn == 0.0) ? 0.0 : sqrt(norm2(s, N)) / bn;
    *iters_out = it;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return status;
}

/* c = W^H z for k columns W[i] (each N complex), z one vector; out k complex. */
void o2_project(const double *Wd, int k, const double *zd, long N, double *outd) {
    const cplx *W = (const cplx *)Wd;
    const cplx *z = (const cplx *)zd;
    cplx *out = (cplx *)outd;
    for (int i = 0; i < k; i++) out[i] = dotc(W + (long)i * N, z, N);
}

int o2_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * FP64 CPU oracle for the propagators of "Temporal blocking of
 * finite-difference stencil operators with sparse off-the-grid sources"
 * (Bisbas et al., arXiv 2010.10248).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file: it exists so that tests, the smoke check and the CPU leg of the
 * benchmark can compare the GPU library against a plain, slow, obviously
 * correct definition. It shares no code, header, table or constant with the
 * GPU library.
 *
 * What it computes is the naive order of the paper's typical time loop
 * (Section I, the first listing): per time step a full stencil sweep over the
 * grid, then a loop over sources scattering their wavelet values to the grid
 * points around each off-grid position, then receiver interpolation. No
 * tiling, no inspector, no fused injection. FP64 throughout, plain loops, an
 * OpenMP split over the outermost x loop only. Zero-Dirichlet outer boundary
 * is implemented by zero-padded copies of every field (a halo of width r).
 *
 * Readings of points where the paper is silent (all listed in the design
 * notes): standard centred Taylor/Fornberg FD weights; leapfrog in time; a
 * damping term m*d(x)*u_t, centred in time, with a quadratic Collino-Tsogka
 * profile inside the stated grid; trilinear injection and interpolation with
 * zero-weight corners dropped; injection of q_s(t_n)*W*dt^2/m into u^{n+1}
 * (Section III-A, the symbolic listing); receivers read the current level u^n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ERANGE -2
#define OR_ENOMEM -3

typedef int64_t i64;

/* ------------------------------------------------------------------------- */
/* Finite-difference weights: Fornberg (1988), "Generation of finite          */
/* difference formulas on arbitrarily spaced grids", Math. Comp. 51.          */
/* c[k][j] is the weight of node x[j] for the k-th derivative at x0.          */
/* ------------------------------------------------------------------------- */
int or_fornberg(int mderiv, int npts, const double *x, double x0, double *out)
{
    if (mderiv < 0 || npts < 1 || mderiv >= npts) return OR_EINVAL;
    int M = mderiv;
    double *c = calloc((size_t)(M + 1) * npts, sizeof(double));
    if (!c) return OR_ENOMEM;
#define C(k, j) c[(size_t)(k) * npts + (j)]
    double c1 = 1.0, c4 = x[0] - x0;
    C(0, 0) = 1.0;
    for (int i = 1; i < npts; i++) {
        int mn = i < M ? i : M;
        double c2 = 1.0, c5 = c4;
        c4 = x[i] - x0;
        for (int j = 0; j < i; j++) {
            double c3 = x[i] - x[j];
            c2 = c2 * c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; k--)
                    C(k, i) = c1 * (k * C(k - 1, i - 1) - c5 * C(k, i - 1)) / c2;
                C(0, i) = -c1 * c5 * C(0, i - 1) / c2;
            }
            for (int k = mn; k >= 1; k--)
                C(k, j) = (c4 * C(k, j) - k * C(k - 1, j)) / c3;
            C(0, j) = c4 * C(0, j) / c3;
        }
        c1 = c2;
    }
    for (int j = 0; j < npts; j++) out[j] = C(M, j);
#undef C
    free(c);
    return OR_OK;
}

/* Centred second derivative of order so on unit spacing: w[0..r], r = so/2,
 * w[j] is the weight of offsets +j and -j. */
int or_weights_d2(int so, double *w)
{
    if (so < 2 || so % 2) return OR_EINVAL;
    int r = so / 2, n = 2 * r + 1;
    double x[64], c[64];
    for (int j = 0; j < n; j++) x[j] = (double)(j - r);
    int st = or_fornberg(2, n, x, 0.0, c);
    if (st) return st;
    for (int j = 0; j <= r; j++) w[j] = c[r + j];
    return OR_OK;
}

/* Centred first derivative of order so on unit spacing: w[0..r-1] is the
 * weight of offset +(j+1); offset -(j+1) has weight -w[j]. */
int or_weights_d1(int so, double *w)
{
    if (so < 2 || so % 2) return OR_EINVAL;
    int r = so / 2, n = 2 * r + 1;
    double x[64], c[64];
    for (int j = 0; j < n; j++) x[j] = (double)(j - r);
    int st = or_fornberg(1, n, x, 0.0, c);
    if (st) return st;
    for (int j = 0; j < r; j++) w[j] = c[r + 1 + j];
    return OR_OK;
}

/* Staggered first derivative of order so: nodes at +-(j+1/2); w[j] is the
 * weight of +(j+1/2), and -(j+1/2) has weight -w[j]. */
int or_weights_d1_staggered(int so, double *w)
{
    if (so < 2 || so % 2) return OR_EINVAL;
    int r = so / 2, n = 2 * r;
    double x[64], c[64];
    for (int j = 0; j < n; j++) x[j] = (double)(j - r) + 0.5;
    int st = or_fornberg(1, n, x, 0.0, c);
    if (st) return st;
    for (int j = 0; j < r; j++) w[j] = c[r + j];
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Trilinear support of an off-grid point (Fig. 3: linear interpolation).    */
/* Corners are enumerated lexicographically in (bx, by, bz), z fastest.       */
/* Returns the number of corners with non-zero weight, or OR_ERANGE.          */
/* ------------------------------------------------------------------------- */
int or_trilinear(const double *p, const double *o, const double *h, const int *n,
                 int *nodes /* [8][3] */, double *w /* [8] */)
{
    int i[3];
    double f[3];
    for (int a = 0; a < 3; a++) {
        double xi = (p[a] - o[a]) / h[a];
        if (!(xi >= 0.0) || !(xi <= (double)(n[a] - 1))) return OR_ERANGE;
        double fl = floor(xi);
        i[a] = (int)fl;
        f[a] = xi - fl;
    }
    int cnt = 0;
    for (int bx = 0; bx < 2; bx++)
        for (int by = 0; by < 2; by++)
            for (int bz = 0; bz < 2; bz++) {
                double wx = bx ? f[0] : 1.0 - f[0];
                double wy = by ? f[1] : 1.0 - f[1];
                double wz = bz ? f[2] : 1.0 - f[2];
                double W = wx * wy * wz;
                if (W == 0.0) continue;
                nodes[3 * cnt + 0] = i[0] + bx;
                nodes[3 * cnt + 1] = i[1] + by;
                nodes[3 * cnt + 2] = i[2] + bz;
                w[cnt] = W;
                cnt++;
            }
    return cnt;
}

/* ------------------------------------------------------------------------- */
/* Damping profile (absorbing layers inside the stated grid, Section IV-B).   */
/* d(i,j,k) = sum_a d0_a (k_a/nbl)^2, k_a the depth into the layer along a,   */
/* d0_a = 3 vmax ln(1/R) / (2 nbl h_a), R = 1e-3.                              */
/* ------------------------------------------------------------------------- */
void or_damping(const int *n, const double *h, int nbl, double vmax, double *d)
{
    const double R = 1e-3;
    for (i64 i = 0; i < n[0]; i++)
        for (i64 j = 0; j < n[1]; j++)
            for (i64 k = 0; k < n[2]; k++) {
                double s = 0.0;
                if (nbl > 0) {
                    i64 idx[3] = {i, j, k};
                    for (int a = 0; a < 3; a++) {
                        i64 lo = nbl - idx[a];
                        i64 hi = idx[a] - (n[a] - 1 - nbl);
                        i64 ka = lo > hi ? lo : hi;
                        if (ka < 0) ka = 0;
                        double d0 = 3.0 * vmax * log(1.0 / R) / (2.0 * nbl * h[a]);
                        double q = (double)ka / (double)nbl;
                        s += d0 * q * q;
                    }
                }
                d[(i * n[1] + j) * n[2] + k] = s;
            }
}

/* ------------------------------------------------------------------------- */
/* Padded field helpers: a field of n[0]*n[1]*n[2] nodes is stored with a     */
/* zero halo of width r on every side, so that every stencil read outside     */
/* [0,n) returns 0 (zero-Dirichlet).                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n[3], r;
    i64 p1, p2; /* padded sizes of axes 1 and 2 */
    i64 total;
} pgrid;

static pgrid pg_make(const int *n, int r)
{
    pgrid g;
    g.n[0] = n[0]; g.n[1] = n[1]; g.n[2] = n[2];
    g.r = r;
    g.p1 = n[1] + 2 * r;
    g.p2 = n[2] + 2 * r;
    g.total = (i64)(n[0] + 2 * r) * g.p1 * g.p2;
    return g;
}

static inline i64 pg_at(const pgrid *g, i64 i, i64 j, i64 k)
{
    return ((i + g->r) * g->p1 + (j + g->r)) * g->p2 + (k + g->r);
}

static void pg_load(const pgrid *g, double *dst, const double *src)
{
    memset(dst, 0, sizeof(double) * g->total);
    for (i64 i = 0; i < g->n[0]; i++)
        for (i64 j = 0; j < g->n[1]; j++)
            for (i64 k = 0; k < g->n[2]; k++)
                dst[pg_at(g, i, j, k)] = src[(i * g->n[1] + j) * g->n[2] + k];
}

static void pg_store(const pgrid *g, double *dst, const double *src)
{
    for (i64 i = 0; i < g->n[0]; i++)
        for (i64 j = 0; j < g->n[1]; j++)
            for (i64 k = 0; k < g->n[2]; k++)
                dst[(i * g->n[1] + j) * g->n[2] + k] = src[pg_at(g, i, j, k)];
}

/* Laplacian of order so: L u = sum_a h_a^-2 sum_{|j|<=r} w_j u(x + j e_a).   */
static double lap_at(const pgrid *g, const double *u, const double *w, const double *h,
                     i64 i, i64 j, i64 k)
{
    int r = g->r;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int q = -r; q <= r; q++) {
        int aq = q < 0 ? -q : q;
        sx += w[aq] * u[pg_at(g, i + q, j, k)];
        sy += w[aq] * u[pg_at(g, i, j + q, k)];
        sz += w[aq] * u[pg_at(g, i, j, k + q)];
    }
    return sx / (h[0] * h[0]) + sy / (h[1] * h[1]) + sz / (h[2] * h[2]);
}

/* Exported Laplacian on an unpadded field (for invariant tests). */
int or_laplacian(const int *n, const double *h, int so, const double *u, double *out)
{
    double w[32];
    if (or_weights_d2(so, w)) return OR_EINVAL;
    pgrid g = pg_make(n, so / 2);
    double *up = malloc(sizeof(double) * g.total);
    if (!up) return OR_ENOMEM;
    pg_load(&g, up, u);
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n[0]; i++)
        for (i64 j = 0; j < n[1]; j++)
            for (i64 k = 0; k < n[2]; k++)
                out[(i * n[1] + j) * n[2] + k] = lap_at(&g, up, w, h, i, j, k);
    free(up);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Isotropic acoustic propagator (Section III-A, equation (acou)):           */
/*   m u_tt + m d u_t - Lap u = sum_s delta(x - x_s) q_s(t),  m = 1/vp^2.     */
/* Leapfrog with c = dt^2/m, alpha = 1 + d dt/2, beta = 1 - d dt/2:           */
/*   u^{n+1} = (c L u^n + 2 u^n - beta u^{n-1}) / alpha                       */
/* then u^{n+1}[node] += W c[node] q_s(t_n) for every source and corner,     */
/* then d^n_r = sum_k W_rk u^n[node_k].                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n[3];
    double h[3], o[3];
    int so, r, nbl;
    double dt;
    double *c;     /* dt^2 vp^2, unpadded */
    double *alpha; /* unpadded */
    double *beta;  /* unpadded */
    double w[32];
} acou;

static int acou_init(acou *A, const int *n, const double *h, const double *o, int so, int nbl,
                     double dt, const double *vp, double vmax_damp)
{
    memcpy(A->n, n, sizeof(int) * 3);
    memcpy(A->h, h, sizeof(double) * 3);
    memcpy(A->o, o, sizeof(double) * 3);
    A->so = so;
    A->r = so / 2;
    A->nbl = nbl;
    A->dt = dt;
    if (or_weights_d2(so, A->w)) return OR_EINVAL;
    i64 N = (i64)n[0] * n[1] * n[2];
    A->c = malloc(sizeof(double) * N);
    A->alpha = malloc(sizeof(double) * N);
    A->beta = malloc(sizeof(double) * N);
    if (!A->c || !A->alpha || !A->beta) return OR_ENOMEM;
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 p = 0; p < N; p++)
            if (vp[p] > vmax) vmax = vp[p];
    }
    or_damping(n, h, nbl, vmax, A->alpha); /* alpha holds d for now */
    for (i64 p = 0; p < N; p++) {
        double d = A->alpha[p];
        A->c[p] = dt * dt * vp[p] * vp[p];
        A->alpha[p] = 1.0 + d * dt / 2.0;
        A->beta[p] = 1.0 - d * dt / 2.0;
    }
    return OR_OK;
}

static void acou_free(acou *A)
{
    free(A->c);
    free(A->alpha);
    free(A->beta);
}

/* One stencil update on padded fields: un = (c L u + 2u - beta up)/alpha.   */
static void acou_stencil(const acou *A, const pgrid *g, double *un, const double *u,
                         const double *up)
{
    const int *n = A->n;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n[0]; i++)
        for (i64 j = 0; j < n[1]; j++)
            for (i64 k = 0; k < n[2]; k++) {
                i64 q = (i * n[1] + j) * n[2] + k;
                i64 p = pg_at(g, i, j, k);
                double L = lap_at(g, u, A->w, A->h, i, j, k);
                un[p] = (A->c[q] * L + 2.0 * u[p] - A->beta[q] * up[p]) / A->alpha[q];
            }
}

/* Scatter sources at time index t into a padded field (first listing, the
 * loop over sources): u[node] += W c[node] q_s(t). */
static int acou_inject(const acou *A, const pgrid *g, double *u, int nsrc, const double *xyz,
                       const double *wav, int t)
{
    for (int s = 0; s < nsrc; s++) {
        int nodes[24];
        double w[8];
        int cnt = or_trilinear(xyz + 3 * s, A->o, A->h, A->n, nodes, w);
        if (cnt < 0) return cnt;
        double q = wav[(i64)t * nsrc + s];
        for (int k = 0; k < cnt; k++) {
            int *nd = nodes + 3 * k;
            i64 qi = ((i64)nd[0] * A->n[1] + nd[1]) * A->n[2] + nd[2];
            u[pg_at(g, nd[0], nd[1], nd[2])] += w[k] * A->c[qi] * q;
        }
    }
    return OR_OK;
}

/* Receiver interpolation from a padded field into out[nrec]. */
static int interp(const int *n, const double *o, const double *h, const pgrid *g, const double *u,
                  int nrec, const double *xyz, double *out)
{
    for (int r = 0; r < nrec; r++) {
        int nodes[24];
        double w[8];
        int cnt = or_trilinear(xyz + 3 * r, o, h, n, nodes, w);
        if (cnt < 0) return cnt;
        double s = 0.0;
        for (int k = 0; k < cnt; k++) {
            int *nd = nodes + 3 * k;
            s += w[k] * u[pg_at(g, nd[0], nd[1], nd[2])];
        }
        out[r] = s;
    }
    return OR_OK;
}

/*
 * Full forward run. Inputs: grid n[3], spacing h[3], origin o[3], space order
 * so (even), sponge width nbl, dt, nt, vp[n0*n1*n2] (m/s), nsrc sources at
 * src_xyz[nsrc][3] with wavelets src_wav[nt][nsrc], nrec receivers at
 * rec_xyz[nrec][3]. vmax_damp > 0 fixes the velocity used by the damping
 * profile (otherwise max(vp)). u0/u1 optionally give u^0 and u^{-1} (NULL =
 * zero initial conditions). Outputs (any may be NULL): traces[nt][nrec] with
 * d^n = P_r u^n, u_last = u^{nt}, u_prev = u^{nt-1}, history[(nt+1)][N]
 * holding u^0..u^{nt}.
 */
int or_acoustic_forward(const int *n, const double *h, const double *o, int so, int nbl,
                        double dt, int nt, const double *vp, double vmax_damp,
                        int nsrc, const double *src_xyz, const double *src_wav,
                        int nrec, const double *rec_xyz,
                        const double *u0, const double *u1,
                        double *traces, double *u_last, double *u_prev, double *history)
{
    acou A;
    int st = acou_init(&A, n, h, o, so, nbl, dt, vp, vmax_damp);
    if (st) return st;
    pgrid g = pg_make(n, A.r);
    i64 N = (i64)n[0] * n[1] * n[2];
    double *a = calloc(g.total, sizeof(double)); /* u^{n-1} */
    double *b = calloc(g.total, sizeof(double)); /* u^n     */
    double *cbuf = calloc(g.total, sizeof(double)); /* u^{n+1} */
    if (!a || !b || !cbuf) { st = OR_ENOMEM; goto done; }
    if (u0) pg_load(&g, b, u0);
    if (u1) pg_load(&g, a, u1);
    if (history) pg_store(&g, history, b);
    for (int t = 0; t < nt; t++) {
        acou_stencil(&A, &g, cbuf, b, a);
        st = acou_inject(&A, &g, cbuf, nsrc, src_xyz, src_wav, t);
        if (st) goto done;
        if (traces) {
            st = interp(n, o, h, &g, b, nrec, rec_xyz, traces + (i64)t * nrec);
            if (st) goto done;
        }
        double *tmp = a; a = b; b = cbuf; cbuf = tmp;
        if (history) pg_store(&g, history + (i64)(t + 1) * N, b);
    }
    if (u_last) pg_store(&g, u_last, b);
    if (u_prev) pg_store(&g, u_prev, a);
done:
    free(a); free(b); free(cbuf);
    acou_free(&A);
    return st;
}

/* Increment of the source loop at time index t applied to a zero grid: the
 * direct per-source scatter that the inspector's decomposition must equal. */
int or_acoustic_inject_increment(const int *n, const double *h, const double *o, int so,
                                 double dt, const double *vp, int nsrc, const double *src_xyz,
                                 const double *src_wav, int t, double *out)
{
    acou A;
    int st = acou_init(&A, n, h, o, so, 0, dt, vp, 1.0);
    if (st) return st;
    pgrid g = pg_make(n, A.r);
    double *u = calloc(g.total, sizeof(double));
    if (!u) { acou_free(&A); return OR_ENOMEM; }
    st = acou_inject(&A, &g, u, nsrc, src_xyz, src_wav, t);
    if (!st) pg_store(&g, out, u);
    free(u);
    acou_free(&A);
    return st;
}

/*
 * Exact discrete adjoint of the forward recursion above, and the gradient of
 * J = 1/2 sum_{k=0}^{nt-1} |P_r u^k - dobs^k|^2 with respect to m = 1/vp^2
 * (the damping profile held fixed). Writing the forward as
 *   u^k = (c/alpha) L u^{k-1} + (2/alpha) u^{k-1} - (beta/alpha) u^{k-2} + s^{k-1},
 *   s^n = c P_s^T q^n,
 * the multiplier in the variable nu = c lambda/alpha obeys the same update
 * backwards in time:
 *   nu^{nt} = nu^{nt+1} = 0,
 *   nu^k = (c/alpha) L nu^{k+1} + (2/alpha) nu^{k+1} - (beta/alpha) nu^{k+2}
 *          + (c/alpha) P_r^T res^k,     k = nt-1 .. 0,
 * and
 *   g = -(1/dt^2) sum_{k=1}^{nt-1} nu^k (c L u^{k-1} + alpha s^{k-1}),
 *   qhat_s^n = P_s (alpha nu^{n+1})   (adjoint of the linear map q -> d).
 *
 * res[nt][nrec] is the data-space vector driving the adjoint (the residual
 * for a gradient, any d' for a dot test). Outputs (NULL to skip):
 * grad[N] (requires u_hist = u^0..u^{nt-1} from the forward), qhat[nt][nsrc],
 * nu1[N] = the adjoint state nu^1.
 */
int or_acoustic_adjoint(const int *n, const double *h, const double *o, int so, int nbl,
                        double dt, int nt, const double *vp, double vmax_damp,
                        int nsrc, const double *src_xyz, const double *src_wav,
                        int nrec, const double *rec_xyz, const double *res,
                        const double *u_hist, double *grad, double *qhat, double *nu1)
{
    acou A;
    int st = acou_init(&A, n, h, o, so, nbl, dt, vp, vmax_damp);
    if (st) return st;
    pgrid g = pg_make(n, A.r);
    i64 N = (i64)n[0] * n[1] * n[2];
    double *a = calloc(g.total, sizeof(double));   /* nu^{k+2} */
    double *b = calloc(g.total, sizeof(double));   /* nu^{k+1} */
    double *cb = calloc(g.total, sizeof(double));  /* nu^k     */
    double *inj = calloc(g.total, sizeof(double)); /* scratch  */
    double *up = grad ? calloc(g.total, sizeof(double)) : NULL;
    if (!a || !b || !cb || !inj || (grad && !up)) { st = OR_ENOMEM; goto done; }
    if (grad) memset(grad, 0, sizeof(double) * N);
    if (qhat) memset(qhat, 0, sizeof(double) * (size_t)nt * nsrc);
    for (int k = nt - 1; k >= 0; k--) {
        /* qhat^{k} = P_s (alpha nu^{k+1}); nu^{k+1} is b. */
        if (qhat) {
            for (int s = 0; s < nsrc; s++) {
                int nodes[24];
                double w[8];
                int cnt = or_trilinear(src_xyz + 3 * s, o, h, n, nodes, w);
                if (cnt < 0) { st = cnt; goto done; }
                double acc = 0.0;
                for (int q = 0; q < cnt; q++) {
                    int *nd = nodes + 3 * q;
                    i64 qi = ((i64)nd[0] * n[1] + nd[1]) * n[2] + nd[2];
                    acc += w[q] * A.alpha[qi] * b[pg_at(&g, nd[0], nd[1], nd[2])];
                }
                qhat[(i64)k * nsrc + s] = acc;
            }
        }
        /* Stencil part of the adjoint update. */
        acou_stencil(&A, &g, cb, b, a);
        /* Residual injection: (c/alpha) P_r^T res^k. */
        for (int r = 0; r < nrec; r++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(rec_xyz + 3 * r, o, h, n, nodes, w);
            if (cnt < 0) { st = cnt; goto done; }
            double rv = res[(i64)k * nrec + r];
            for (int q = 0; q < cnt; q++) {
                int *nd = nodes + 3 * q;
                i64 qi = ((i64)nd[0] * n[1] + nd[1]) * n[2] + nd[2];
                cb[pg_at(&g, nd[0], nd[1], nd[2])] += A.c[qi] / A.alpha[qi] * w[q] * rv;
            }
        }
        /* cb = nu^k. Gradient term for k >= 1 uses u^{k-1} and s^{k-1}. */
        if (grad && k >= 1) {
            pg_load(&g, up, u_hist + (i64)(k - 1) * N);
            memset(inj, 0, sizeof(double) * g.total);
            st = acou_inject(&A, &g, inj, nsrc, src_xyz, src_wav, k - 1);
            if (st) goto done;
#pragma omp parallel for schedule(static)
            for (i64 i = 0; i < n[0]; i++)
                for (i64 j = 0; j < n[1]; j++)
                    for (i64 kk = 0; kk < n[2]; kk++) {
                        i64 q = (i * n[1] + j) * n[2] + kk;
                        i64 p = pg_at(&g, i, j, kk);
                        double Lu = lap_at(&g, up, A.w, A.h, i, j, kk);
                        grad[q] += cb[p] * (A.c[q] * Lu + A.alpha[q] * inj[p]);
                    }
        }
        double *tmp = a; a = b; b = cb; cb = tmp;
        /* now b = nu^k, a = nu^{k+1} */
        if (k == 1 && nu1) pg_store(&g, nu1, b);
    }
    if (grad)
        for (i64 q = 0; q < N; q++) grad[q] *= -1.0 / (dt * dt);
done:
    free(a); free(b); free(cb); free(inj); free(up);
    acou_free(&A);
    return st;
}

/* Objective J = 1/2 sum_k |d^k - dobs^k|^2 (FP64, k ascending, r ascending). */
double or_misfit(int nt, int nrec, const double *d, const double *dobs, double *res)
{
    double J = 0.0;
    for (i64 i = 0; i < (i64)nt * nrec; i++) {
        double r = d[i] - dobs[i];
        if (res) res[i] = r;
        J += 0.5 * r * r;
    }
    return J;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

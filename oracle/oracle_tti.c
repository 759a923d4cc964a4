/*
 * FP64 CPU oracle of the pseudo-acoustic TTI propagator (Section III-B of
 * "Temporal blocking of finite-difference stencil operators with sparse
 * off-the-grid sources", Bisbas et al., arXiv 2010.10248).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product path may
 * link, load or call it; it shares nothing with the GPU library.
 *
 * The paper defines the rotated operators only through the first one
 * (G_xbar = D_xbar^T D_xbar with the rotated derivative of its Section III-B)
 * and cites the self-adjoint pseudo-acoustic system for the rest. Reading
 * used here (listed in the design notes):
 *   a   = (sin t cos f, sin t sin f, cos t)      the symmetry axis (t = theta
 *         tilt from vertical, f = phi azimuth), completing the frame of the
 *         paper's D_xbar;
 *   D u = sum_a a_a d_a u                         centred first derivatives
 *         of the space order, every field and intermediate zero outside the
 *         grid, so that
 *   Hz u = sum_b d_b (a_b D u) = -D^T D u        exactly;
 *   H0 u = L u - Hz u                             L the centred Laplacian;
 *   m p_tt + m d p_t = (1+2 eps) H0 p + sqrt(1+2 del) Hz r
 *   m r_tt + m d r_t = sqrt(1+2 del) H0 p + Hz r, with del := min(del, eps).
 * Time stepping, damping, injection (the same W dt^2/m q into p and r) and
 * receivers (reading p^n) follow the acoustic oracle. Naive order per step:
 * the operators and both updates at every node, then injection, then
 * interpolation of the current level.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3

int or_weights_d1(int so, double *w);
int or_weights_d2(int so, double *w);
int or_trilinear(const double *p, const double *o, const double *h, const int *n, int *nodes,
                 double *w);
void or_damping(const int *n, const double *h, int nbl, double vmax, double *d);

typedef struct {
    int n[3], r;
    double h[3];
    double w1[16], w2[17];
} tgrid;

static inline double at(const tgrid *G, const double *u, i64 i, i64 j, i64 k)
{
    if (i < 0 || j < 0 || k < 0 || i >= G->n[0] || j >= G->n[1] || k >= G->n[2]) return 0.0;
    return u[(i * G->n[1] + j) * G->n[2] + k];
}

/* Centred first derivative of u along axis ax at node (i, j, k). */
static double d1(const tgrid *G, const double *u, i64 i, i64 j, i64 k, int ax)
{
    double s = 0.0;
    for (int m = 1; m <= G->r; m++) {
        i64 di = ax == 0 ? m : 0, dj = ax == 1 ? m : 0, dk = ax == 2 ? m : 0;
        s += G->w1[m - 1] * (at(G, u, i + di, j + dj, k + dk) - at(G, u, i - di, j - dj, k - dk));
    }
    return s / G->h[ax];
}

/* Centred Laplacian of u at node (i, j, k). */
static double lap(const tgrid *G, const double *u, i64 i, i64 j, i64 k)
{
    double s = 0.0;
    const double c = at(G, u, i, j, k);
    for (int ax = 0; ax < 3; ax++) {
        double a = G->w2[0] * c;
        for (int m = 1; m <= G->r; m++) {
            i64 di = ax == 0 ? m : 0, dj = ax == 1 ? m : 0, dk = ax == 2 ? m : 0;
            a += G->w2[m] * (at(G, u, i + di, j + dj, k + dk) + at(G, u, i - di, j - dj, k - dk));
        }
        s += a / (G->h[ax] * G->h[ax]);
    }
    return s;
}

static int tgrid_init(tgrid *G, const int *n, const double *h, int so)
{
    memcpy(G->n, n, sizeof(int) * 3);
    memcpy(G->h, h, sizeof(double) * 3);
    G->r = so / 2;
    if (so < 2 || so > 16 || so % 2) return OR_EINVAL;
    if (or_weights_d1(so, G->w1) || or_weights_d2(so, G->w2)) return OR_EINVAL;
    return OR_OK;
}

/* Hz u into out, with the axis components ax/ay/az per node and three
 * scratch fields (each N). */
static void apply_hz(const tgrid *G, const double *ax, const double *ay, const double *az,
                     const double *u, double *out, double *wx, double *wy, double *wz)
{
    const i64 n0 = G->n[0], n1 = G->n[1], n2 = G->n[2];
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n0; i++)
        for (i64 j = 0; j < n1; j++)
            for (i64 k = 0; k < n2; k++) {
                i64 q = (i * n1 + j) * n2 + k;
                double Du = ax[q] * d1(G, u, i, j, k, 0) + ay[q] * d1(G, u, i, j, k, 1) +
                            az[q] * d1(G, u, i, j, k, 2);
                wx[q] = ax[q] * Du;
                wy[q] = ay[q] * Du;
                wz[q] = az[q] * Du;
            }
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n0; i++)
        for (i64 j = 0; j < n1; j++)
            for (i64 k = 0; k < n2; k++) {
                i64 q = (i * n1 + j) * n2 + k;
                out[q] = d1(G, wx, i, j, k, 0) + d1(G, wy, i, j, k, 1) + d1(G, wz, i, j, k, 2);
            }
}

static void axis_of(const double *theta, const double *phi, i64 N, double *ax, double *ay,
                    double *az)
{
    for (i64 q = 0; q < N; q++) {
        ax[q] = sin(theta[q]) * cos(phi[q]);
        ay[q] = sin(theta[q]) * sin(phi[q]);
        az[q] = cos(theta[q]);
    }
}

/*
 * The spatial operators alone, for checking them: lap_out = L u and
 * hz_out = Hz u (either may be NULL).
 */
int or_tti_operators(const int *n, const double *h, int so, const double *theta,
                     const double *phi, const double *u, double *lap_out, double *hz_out)
{
    tgrid G;
    int st = tgrid_init(&G, n, h, so);
    if (st) return st;
    const i64 N = (i64)n[0] * n[1] * n[2];
    double *buf = malloc(sizeof(double) * 6 * N);
    if (!buf) return OR_ENOMEM;
    double *ax = buf, *ay = buf + N, *az = buf + 2 * N;
    axis_of(theta, phi, N, ax, ay, az);
    if (hz_out) apply_hz(&G, ax, ay, az, u, hz_out, buf + 3 * N, buf + 4 * N, buf + 5 * N);
    if (lap_out) {
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n[0]; i++)
            for (i64 j = 0; j < n[1]; j++)
                for (i64 k = 0; k < n[2]; k++)
                    lap_out[(i * n[1] + j) * n[2] + k] = lap(&G, u, i, j, k);
    }
    free(buf);
    return OR_OK;
}

static int scatter(const tgrid *G, const double *o, double *u, const double *c, int nsrc,
                   const double *xyz, const double *wav, int t)
{
    for (int s = 0; s < nsrc; s++) {
        int nodes[24];
        double w[8];
        int cnt = or_trilinear(xyz + 3 * s, o, G->h, G->n, nodes, w);
        if (cnt < 0) return cnt;
        const double q = wav[(i64)t * nsrc + s];
        for (int k = 0; k < cnt; k++) {
            const i64 qi = ((i64)nodes[3 * k] * G->n[1] + nodes[3 * k + 1]) * G->n[2] +
                           nodes[3 * k + 2];
            u[qi] += w[k] * c[qi] * q;
        }
    }
    return OR_OK;
}

static int gather(const tgrid *G, const double *o, const double *u, int nrec, const double *xyz,
                  double *out)
{
    for (int r = 0; r < nrec; r++) {
        int nodes[24];
        double w[8];
        int cnt = or_trilinear(xyz + 3 * r, o, G->h, G->n, nodes, w);
        if (cnt < 0) return cnt;
        double s = 0.0;
        for (int k = 0; k < cnt; k++)
            s += w[k] * u[((i64)nodes[3 * k] * G->n[1] + nodes[3 * k + 1]) * G->n[2] +
                          nodes[3 * k + 2]];
        out[r] = s;
    }
    return OR_OK;
}

/*
 * Forward run from zero state. Inputs as or_acoustic_forward plus eps, del,
 * theta, phi [N]. Outputs (any may be NULL): traces[nt][nrec] (d^n = P_r p^n),
 * p^{nt}, p^{nt-1}, r^{nt}, r^{nt-1}, and the histories p^0..p^{nt-1},
 * r^0..r^{nt-1} ([nt][N] each) for the gradient.
 */
int or_tti_forward(const int *n, const double *h, const double *o, int so, int nbl, double dt,
                   int nt, const double *vp, const double *eps, const double *del,
                   const double *theta, const double *phi, double vmax_damp, int nsrc,
                   const double *src_xyz, const double *src_wav, int nrec, const double *rec_xyz,
                   double *traces, double *p_last, double *p_prev, double *r_last,
                   double *r_prev, double *p_hist, double *r_hist)
{
    tgrid G;
    int st = tgrid_init(&G, n, h, so);
    if (st) return st;
    const i64 N = (i64)n[0] * n[1] * n[2];
    const int NB = 16;
    double *buf = calloc((size_t)NB * N, sizeof(double));
    if (!buf) return OR_ENOMEM;
    double *ax = buf, *ay = buf + N, *az = buf + 2 * N;
    double *c = buf + 3 * N, *alpha = buf + 4 * N, *beta = buf + 5 * N;
    double *e1 = buf + 6 * N, *sd = buf + 7 * N;
    double *p0 = buf + 8 * N, *p1 = buf + 9 * N, *p2 = buf + 10 * N; /* p^{n-1}, p^n, p^{n+1} */
    double *r0 = buf + 11 * N, *r1 = buf + 12 * N, *r2 = buf + 13 * N;
    double *hzp = buf + 14 * N, *hzr = buf + 15 * N;
    double *wx = malloc(sizeof(double) * 3 * N);
    if (!wx) {
        free(buf);
        return OR_ENOMEM;
    }
    double *wy = wx + N, *wz = wx + 2 * N;
    axis_of(theta, phi, N, ax, ay, az);
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 q = 0; q < N; q++)
            if (vp[q] > vmax) vmax = vp[q];
    }
    or_damping(n, h, nbl, vmax, alpha); /* alpha holds d for now */
    for (i64 q = 0; q < N; q++) {
        const double d = alpha[q];
        c[q] = dt * dt * vp[q] * vp[q];
        alpha[q] = 1.0 + d * dt / 2.0;
        beta[q] = 1.0 - d * dt / 2.0;
        const double dl = del[q] < eps[q] ? del[q] : eps[q];
        e1[q] = 1.0 + 2.0 * eps[q];
        sd[q] = sqrt(1.0 + 2.0 * dl);
    }
    for (int t = 0; t < nt; t++) {
        if (p_hist) memcpy(p_hist + (i64)t * N, p1, sizeof(double) * N);
        if (r_hist) memcpy(r_hist + (i64)t * N, r1, sizeof(double) * N);
        apply_hz(&G, ax, ay, az, p1, hzp, wx, wy, wz);
        apply_hz(&G, ax, ay, az, r1, hzr, wx, wy, wz);
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n[0]; i++)
            for (i64 j = 0; j < n[1]; j++)
                for (i64 k = 0; k < n[2]; k++) {
                    const i64 q = (i * n[1] + j) * n[2] + k;
                    const double h0p = lap(&G, p1, i, j, k) - hzp[q];
                    const double rp = e1[q] * h0p + sd[q] * hzr[q];
                    const double rr = sd[q] * h0p + hzr[q];
                    p2[q] = (c[q] * rp + 2.0 * p1[q] - beta[q] * p0[q]) / alpha[q];
                    r2[q] = (c[q] * rr + 2.0 * r1[q] - beta[q] * r0[q]) / alpha[q];
                }
        if ((st = scatter(&G, o, p2, c, nsrc, src_xyz, src_wav, t))) goto done;
        if ((st = scatter(&G, o, r2, c, nsrc, src_xyz, src_wav, t))) goto done;
        if (traces && (st = gather(&G, o, p1, nrec, rec_xyz, traces + (i64)t * nrec))) goto done;
        double *tp = p0;
        p0 = p1;
        p1 = p2;
        p2 = tp;
        tp = r0;
        r0 = r1;
        r1 = r2;
        r2 = tp;
    }
    if (p_last) memcpy(p_last, p1, sizeof(double) * N);
    if (p_prev) memcpy(p_prev, p0, sizeof(double) * N);
    if (r_last) memcpy(r_last, r1, sizeof(double) * N);
    if (r_prev) memcpy(r_prev, r0, sizeof(double) * N);
done:
    free(wx);
    free(buf);
    return st;
}

/*
 * Exact discrete adjoint of the linear map q -> d of or_tti_forward. With
 * w = (p, r), the forward is
 *   w^k = (c/alpha) A w^{k-1} + (2/alpha) w^{k-1} - (beta/alpha) w^{k-2} + s^{k-1},
 *   A = [[e H0, s Hz], [s H0, Hz]] = D H,  D = [[e, s], [s, 1]] per node,
 *   H = diag(H0, Hz),  s^n = c P_s^T q^n added to both fields,  d^k = P_r p^k,
 * with e = 1 + 2 eps, s = sqrt(1 + 2 min(del, eps)). H0 and Hz are symmetric
 * (Hz = -D^T D with zero outside the grid; L symmetric), so A^T = H D, and
 * the multiplier obeys, backwards from lambda^{nt} = lambda^{nt+1} = 0,
 *   y = (c/alpha) lambda^{k+1}
 *   lambda^k = H (D y) + (2/alpha) lambda^{k+1} - (beta/alpha) lambda^{k+2}
 *              + (P_r^T res^k, 0),                           k = nt-1 .. 0,
 * and the adjoint of the source map is
 *   qhat_s^n = P_s (c (lambda_p^{n+1} + lambda_r^{n+1})).
 * res[nt][nrec] is any data-space vector; output qhat[nt][nsrc].
 *
 * With the forward histories p_hist, r_hist ([nt][N], levels 0..nt-1) and
 * the wavelets src_wav, grad[N] receives the gradient with respect to
 * m = 1/vp^2 of J = 1/2 sum_k |P_r p^k - dobs^k|^2 when res = P_r p - dobs
 * (eps, delta, the axis and the damping held fixed). Differentiating the
 * alpha-scaled forward equation, where c = dt^2/m enters A w^{k-1} and the
 * injection c P_s^T q^{k-1}, gives
 *   grad = -(1/dt^2) sum_{k=1}^{nt-1} sum_{f = p, r} y_f^k (c (A w^{k-1})_f + alpha s^{k-1}),
 *   y^k = (c/alpha) lambda^k,  s^{k-1} = c P_s^T q^{k-1},
 * the acoustic formula with the coupled operator.
 */
int or_tti_adjoint(const int *n, const double *h, const double *o, int so, int nbl, double dt,
                   int nt, const double *vp, const double *eps, const double *del,
                   const double *theta, const double *phi, double vmax_damp, int nsrc,
                   const double *src_xyz, const double *src_wav, int nrec, const double *rec_xyz,
                   const double *res, const double *p_hist, const double *r_hist, double *grad,
                   double *qhat)
{
    tgrid G;
    int st = tgrid_init(&G, n, h, so);
    if (st) return st;
    const i64 N = (i64)n[0] * n[1] * n[2];
    const int NB = 21;
    if (grad && (!p_hist || !r_hist || !src_wav)) return OR_EINVAL;
    double *buf = calloc((size_t)NB * N, sizeof(double));
    if (!buf) return OR_ENOMEM;
    double *ax = buf, *ay = buf + N, *az = buf + 2 * N;
    double *c = buf + 3 * N, *alpha = buf + 4 * N, *beta = buf + 5 * N;
    double *e1 = buf + 6 * N, *sd = buf + 7 * N;
    double *p0 = buf + 8 * N, *p1 = buf + 9 * N, *p2 = buf + 10 * N; /* lambda_p k+2, k+1, k */
    double *r0 = buf + 11 * N, *r1 = buf + 12 * N, *r2 = buf + 13 * N;
    double *zp = buf + 14 * N, *zr = buf + 15 * N, *hzp = buf + 16 * N, *hzr = buf + 17 * N;
    double *hfp = buf + 18 * N, *hfr = buf + 19 * N, *sk = buf + 20 * N; /* Hz p^k, Hz r^k, s^k */
    double *wx = malloc(sizeof(double) * 3 * N);
    if (!wx) {
        free(buf);
        return OR_ENOMEM;
    }
    double *wy = wx + N, *wz = wx + 2 * N;
    axis_of(theta, phi, N, ax, ay, az);
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 q = 0; q < N; q++)
            if (vp[q] > vmax) vmax = vp[q];
    }
    or_damping(n, h, nbl, vmax, alpha); /* alpha holds d for now */
    for (i64 q = 0; q < N; q++) {
        const double d = alpha[q];
        c[q] = dt * dt * vp[q] * vp[q];
        alpha[q] = 1.0 + d * dt / 2.0;
        beta[q] = 1.0 - d * dt / 2.0;
        const double dl = del[q] < eps[q] ? del[q] : eps[q];
        e1[q] = 1.0 + 2.0 * eps[q];
        sd[q] = sqrt(1.0 + 2.0 * dl);
    }
    if (qhat) memset(qhat, 0, sizeof(double) * (size_t)nt * nsrc);
    if (grad) memset(grad, 0, sizeof(double) * N);
    for (int k = nt - 1; k >= 0; k--) {
        /* Gradient term of level k+1: y^{k+1} = (c/alpha) lambda^{k+1} against
         * c A w^k + alpha s^k, for k <= nt-2 (lambda^{nt} = 0). */
        if (grad && k <= nt - 2) {
            const double *pk = p_hist + (i64)k * N, *rk = r_hist + (i64)k * N;
            apply_hz(&G, ax, ay, az, pk, hfp, wx, wy, wz);
            apply_hz(&G, ax, ay, az, rk, hfr, wx, wy, wz);
            memset(sk, 0, sizeof(double) * N);
            if ((st = scatter(&G, o, sk, c, nsrc, src_xyz, src_wav, k))) goto done;
#pragma omp parallel for schedule(static)
            for (i64 i = 0; i < n[0]; i++)
                for (i64 j = 0; j < n[1]; j++)
                    for (i64 kk = 0; kk < n[2]; kk++) {
                        const i64 q = (i * n[1] + j) * n[2] + kk;
                        const double h0 = lap(&G, pk, i, j, kk) - hfp[q];
                        const double ap = e1[q] * h0 + sd[q] * hfr[q];
                        const double ar = sd[q] * h0 + hfr[q];
                        const double yp = c[q] / alpha[q] * p1[q], yr = c[q] / alpha[q] * r1[q];
                        grad[q] += yp * (c[q] * ap + alpha[q] * sk[q]) +
                                   yr * (c[q] * ar + alpha[q] * sk[q]);
                    }
        }
        /* qhat^k from lambda^{k+1}. */
        for (int s = 0; qhat && s < nsrc; s++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(src_xyz + 3 * s, o, G.h, G.n, nodes, w);
            if (cnt < 0) {
                st = cnt;
                goto done;
            }
            double acc = 0.0;
            for (int q = 0; q < cnt; q++) {
                const i64 qi = ((i64)nodes[3 * q] * n[1] + nodes[3 * q + 1]) * n[2] +
                               nodes[3 * q + 2];
                acc += w[q] * c[qi] * (p1[qi] + r1[qi]);
            }
            qhat[(i64)k * nsrc + s] = acc;
        }
        /* D y with y = (c/alpha) lambda^{k+1}. */
        for (i64 q = 0; q < N; q++) {
            const double yp = c[q] / alpha[q] * p1[q], yr = c[q] / alpha[q] * r1[q];
            zp[q] = e1[q] * yp + sd[q] * yr;
            zr[q] = sd[q] * yp + yr;
        }
        apply_hz(&G, ax, ay, az, zp, hzp, wx, wy, wz);
        apply_hz(&G, ax, ay, az, zr, hzr, wx, wy, wz);
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n[0]; i++)
            for (i64 j = 0; j < n[1]; j++)
                for (i64 kk = 0; kk < n[2]; kk++) {
                    const i64 q = (i * n[1] + j) * n[2] + kk;
                    const double h0 = lap(&G, zp, i, j, kk) - hzp[q];
                    p2[q] = h0 + (2.0 * p1[q] - beta[q] * p0[q]) / alpha[q];
                    r2[q] = hzr[q] + (2.0 * r1[q] - beta[q] * r0[q]) / alpha[q];
                }
        /* Residual: (P_r^T res^k) into the p component. */
        for (int rr = 0; rr < nrec; rr++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(rec_xyz + 3 * rr, o, G.h, G.n, nodes, w);
            if (cnt < 0) {
                st = cnt;
                goto done;
            }
            const double rv = res[(i64)k * nrec + rr];
            for (int q = 0; q < cnt; q++)
                p2[((i64)nodes[3 * q] * n[1] + nodes[3 * q + 1]) * n[2] + nodes[3 * q + 2]] +=
                    w[q] * rv;
        }
        double *tp = p0;
        p0 = p1;
        p1 = p2;
        p2 = tp;
        tp = r0;
        r0 = r1;
        r1 = r2;
        r2 = tp;
    }
    if (grad)
        for (i64 q = 0; q < N; q++) grad[q] *= -1.0 / (dt * dt);
done:
    free(wx);
    free(buf);
    return st;
}

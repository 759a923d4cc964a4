/*
 * FP64 CPU oracle of the isotropic elastic velocity-stress propagator
 * (Section III-C of "Temporal blocking of finite-difference stencil operators
 * with sparse off-the-grid sources", Bisbas et al., arXiv 2010.10248).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c.
 *
 * The paper gives the first-order system (its elastic equations) and leaves
 * the discretisation open. Reading used here (listed in the design notes):
 *  - Staggered grid: txx, tyy, tzz at nodes (i, j, k); vx at (i+1/2, j, k),
 *    vy at (i, j+1/2, k), vz at (i, j, k+1/2); txy at (i+1/2, j+1/2, k),
 *    txz at (i+1/2, j, k+1/2), tyz at (i, j+1/2, k+1/2); all arrays n^3, the
 *    element [i][j][k] at the node index plus the component's half offsets.
 *  - Staggered first derivatives of the space order (weights of +-(m+1/2)),
 *    every field zero outside the grid.
 *  - b = 1/rho, mu = rho vs^2, lambda = rho (vp^2 - 2 vs^2) at nodes; b at a
 *    velocity point is the mean of its 2 neighbouring nodes, mu at a shear
 *    point the mean of its 4 neighbouring nodes (a neighbour outside the grid
 *    takes the value of the nearest node inside).
 *  - Step n from (v^{n-1/2}, t^n), damping d at the element's node index:
 *      v^{n+1/2} = (beta v^{n-1/2} + dt b (div t^n)) / alpha
 *      t^{n+1}   = (beta t^n + dt (lambda tr(grad v) I + mu (grad v + grad v^T))) / alpha
 *      t_ii^{n+1} += dt W q(t_n)       (explosive source, i = x, y, z)
 *  - Receivers read the current levels: vz^{n-1/2} (trilinear on the vz grid,
 *    whose origin is shifted by h/2 in z) and P^n = (txx + tyy + tzz)^n / 3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3

int or_weights_d1_staggered(int so, double *w);
int or_trilinear(const double *p, const double *o, const double *h, const int *n, int *nodes,
                 double *w);
void or_damping(const int *n, const double *h, int nbl, double vmax, double *d);

enum { VX, VY, VZ, TXX, TYY, TZZ, TXY, TXZ, TYZ, NF };

typedef struct {
    int n[3], r;
    double h[3];
    double w[8];
} egrid;

static inline i64 idx(const egrid *G, i64 i, i64 j, i64 k)
{
    return (i * G->n[1] + j) * G->n[2] + k;
}

static inline double at(const egrid *G, const double *u, i64 i, i64 j, i64 k)
{
    if (i < 0 || j < 0 || k < 0 || i >= G->n[0] || j >= G->n[1] || k >= G->n[2]) return 0.0;
    return u[idx(G, i, j, k)];
}

/* Staggered derivative along axis ax at element (i, j, k). fwd = 1: the field
 * sits at integer positions along ax and the target half a cell above
 * (samples [i+m+1] - [i-m]); fwd = 0: the field sits half a cell above its
 * index and the target at the integer position (samples [i+m] - [i-m-1]). */
static double dst(const egrid *G, const double *u, i64 i, i64 j, i64 k, int ax, int fwd)
{
    double s = 0.0;
    for (int m = 0; m < G->r; m++) {
        i64 a = fwd ? m + 1 : m, b = fwd ? -m : -m - 1;
        double up = at(G, u, i + (ax == 0 ? a : 0), j + (ax == 1 ? a : 0), k + (ax == 2 ? a : 0));
        double dn = at(G, u, i + (ax == 0 ? b : 0), j + (ax == 1 ? b : 0), k + (ax == 2 ? b : 0));
        s += G->w[m] * (up - dn);
    }
    return s / G->h[ax];
}

static inline double clampv(const egrid *G, const double *p, i64 i, i64 j, i64 k)
{
    i = i < 0 ? 0 : (i >= G->n[0] ? G->n[0] - 1 : i);
    j = j < 0 ? 0 : (j >= G->n[1] ? G->n[1] - 1 : j);
    k = k < 0 ? 0 : (k >= G->n[2] ? G->n[2] - 1 : k);
    return p[idx(G, i, j, k)];
}

static int interp(const egrid *G, const double *o, const double *u, const double *xyz,
                  double *out)
{
    int nodes[24];
    double w[8];
    int cnt = or_trilinear(xyz, o, G->h, G->n, nodes, w);
    if (cnt < 0) return cnt;
    double s = 0.0;
    for (int c = 0; c < cnt; c++) s += w[c] * u[idx(G, nodes[3 * c], nodes[3 * c + 1], nodes[3 * c + 2])];
    *out = s;
    return OR_OK;
}

/* Material parameters at the nodes (b = 1/rho, lambda, mu) and their means:
 * b at the three velocity points (2 nodes), mu at the three shear points
 * (4 nodes, a node beyond the grid taken as the nearest inside one). */
static void set_params(const egrid *G, const double *vp, const double *vs, const double *rho,
                       double *P)
{
    const i64 N = (i64)G->n[0] * G->n[1] * G->n[2];
    double *b = P, *lam = P + N, *mu = P + 2 * N, *bx = P + 3 * N, *by = P + 4 * N,
           *bz = P + 5 * N, *mxy = P + 6 * N, *mxz = P + 7 * N, *myz = P + 8 * N;
    for (i64 q = 0; q < N; q++) {
        b[q] = 1.0 / rho[q];
        mu[q] = rho[q] * vs[q] * vs[q];
        lam[q] = rho[q] * (vp[q] * vp[q] - 2.0 * vs[q] * vs[q]);
    }
    for (i64 i = 0; i < G->n[0]; i++)
        for (i64 j = 0; j < G->n[1]; j++)
            for (i64 k = 0; k < G->n[2]; k++) {
                i64 q = idx(G, i, j, k);
                bx[q] = 0.5 * (clampv(G, b, i, j, k) + clampv(G, b, i + 1, j, k));
                by[q] = 0.5 * (clampv(G, b, i, j, k) + clampv(G, b, i, j + 1, k));
                bz[q] = 0.5 * (clampv(G, b, i, j, k) + clampv(G, b, i, j, k + 1));
                mxy[q] = 0.25 * (clampv(G, mu, i, j, k) + clampv(G, mu, i + 1, j, k) +
                                 clampv(G, mu, i, j + 1, k) + clampv(G, mu, i + 1, j + 1, k));
                mxz[q] = 0.25 * (clampv(G, mu, i, j, k) + clampv(G, mu, i + 1, j, k) +
                                 clampv(G, mu, i, j, k + 1) + clampv(G, mu, i + 1, j, k + 1));
                myz[q] = 0.25 * (clampv(G, mu, i, j, k) + clampv(G, mu, i, j + 1, k) +
                                 clampv(G, mu, i, j, k + 1) + clampv(G, mu, i, j + 1, k + 1));
            }
}

/* Velocity pass in place on F[9][N]: v = (beta v + dt b (div t)) / alpha. */
static void vel_pass(const egrid *G, double *F, const double *P, const double *dmp, double dt)
{
    const i64 N = (i64)G->n[0] * G->n[1] * G->n[2];
    const double *bx = P + 3 * N, *by = P + 4 * N, *bz = P + 5 * N;
    double *vx = F + VX * N, *vy = F + VY * N, *vz = F + VZ * N;
    const double *txx = F + TXX * N, *tyy = F + TYY * N, *tzz = F + TZZ * N;
    const double *txy = F + TXY * N, *txz = F + TXZ * N, *tyz = F + TYZ * N;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < G->n[0]; i++)
        for (i64 j = 0; j < G->n[1]; j++)
            for (i64 k = 0; k < G->n[2]; k++) {
                i64 q = idx(G, i, j, k);
                double al = 1.0 + dmp[q] * dt / 2.0, be = 1.0 - dmp[q] * dt / 2.0;
                double fx = dst(G, txx, i, j, k, 0, 1) + dst(G, txy, i, j, k, 1, 0) +
                            dst(G, txz, i, j, k, 2, 0);
                double fy = dst(G, txy, i, j, k, 0, 0) + dst(G, tyy, i, j, k, 1, 1) +
                            dst(G, tyz, i, j, k, 2, 0);
                double fz = dst(G, txz, i, j, k, 0, 0) + dst(G, tyz, i, j, k, 1, 0) +
                            dst(G, tzz, i, j, k, 2, 1);
                vx[q] = (be * vx[q] + dt * bx[q] * fx) / al;
                vy[q] = (be * vy[q] + dt * by[q] * fy) / al;
                vz[q] = (be * vz[q] + dt * bz[q] * fz) / al;
            }
}

/* Stress pass in place on F[9][N]:
 * t = (beta t + dt (lambda tr(grad v) I + mu (grad v + grad v^T))) / alpha. */
static void str_pass(const egrid *G, double *F, const double *P, const double *dmp, double dt)
{
    const i64 N = (i64)G->n[0] * G->n[1] * G->n[2];
    const double *lam = P + N, *mu = P + 2 * N, *mxy = P + 6 * N, *mxz = P + 7 * N,
                 *myz = P + 8 * N;
    const double *vx = F + VX * N, *vy = F + VY * N, *vz = F + VZ * N;
    double *txx = F + TXX * N, *tyy = F + TYY * N, *tzz = F + TZZ * N;
    double *txy = F + TXY * N, *txz = F + TXZ * N, *tyz = F + TYZ * N;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < G->n[0]; i++)
        for (i64 j = 0; j < G->n[1]; j++)
            for (i64 k = 0; k < G->n[2]; k++) {
                i64 q = idx(G, i, j, k);
                double al = 1.0 + dmp[q] * dt / 2.0, be = 1.0 - dmp[q] * dt / 2.0;
                double exx = dst(G, vx, i, j, k, 0, 0), eyy = dst(G, vy, i, j, k, 1, 0),
                       ezz = dst(G, vz, i, j, k, 2, 0);
                double tr = exx + eyy + ezz;
                txx[q] = (be * txx[q] + dt * (lam[q] * tr + 2.0 * mu[q] * exx)) / al;
                tyy[q] = (be * tyy[q] + dt * (lam[q] * tr + 2.0 * mu[q] * eyy)) / al;
                tzz[q] = (be * tzz[q] + dt * (lam[q] * tr + 2.0 * mu[q] * ezz)) / al;
                double gxy = dst(G, vx, i, j, k, 1, 1) + dst(G, vy, i, j, k, 0, 1);
                double gxz = dst(G, vx, i, j, k, 2, 1) + dst(G, vz, i, j, k, 0, 1);
                double gyz = dst(G, vy, i, j, k, 2, 1) + dst(G, vz, i, j, k, 1, 1);
                txy[q] = (be * txy[q] + dt * mxy[q] * gxy) / al;
                txz[q] = (be * txz[q] + dt * mxz[q] * gxz) / al;
                tyz[q] = (be * tyz[q] + dt * myz[q] * gyz) / al;
            }
}

/*
 * One velocity pass (which & 1) and/or one stress pass (which & 2), in that
 * order, applied in place to a given state F[9][N] (vx vy vz txx tyy tzz txy
 * txz tyz), with the forward's parameters and damping; for checking the two
 * passes on their own against closed forms.
 */
int or_elastic_passes(const int *n, const double *h, int so, int nbl, double dt,
                      const double *vp, const double *vs, const double *rho, double vmax_damp,
                      int which, double *F)
{
    egrid G;
    memcpy(G.n, n, sizeof(int) * 3);
    memcpy(G.h, h, sizeof(double) * 3);
    G.r = so / 2;
    if (so < 2 || so > 16 || so % 2 || or_weights_d1_staggered(so, G.w)) return OR_EINVAL;
    const i64 N = (i64)n[0] * n[1] * n[2];
    double *P = calloc((size_t)10 * N, sizeof(double));
    if (!P) return OR_ENOMEM;
    double *dmp = P + 9 * N;
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 q = 0; q < N; q++)
            if (vp[q] > vmax) vmax = vp[q];
    }
    or_damping(n, h, nbl, vmax, dmp);
    set_params(&G, vp, vs, rho, P);
    if (which & 1) vel_pass(&G, F, P, dmp, dt);
    if (which & 2) str_pass(&G, F, P, dmp, dt);
    free(P);
    return OR_OK;
}

/*
 * Forward run from zero state. traces[2][nt][nrec]: vz then P (either block
 * zero-sized if traces is NULL). state[9][N] (optional): v^{nt-1/2} and
 * t^{nt} in the order vx vy vz txx tyy tzz txy txz tyz. energy[nt]
 * (optional): E^{n+1/2} = 1/2 sum_v |v^{n+1/2}|^2 / b + 1/2 <t^{n+1}, C^-1 t^n>
 * after step n (needs mu > 0 everywhere; exactly conserved by the scheme
 * without damping and source). hist[nt][9][N] (optional, for the gradient):
 * per step t the velocities after its velocity pass, v^{t+1/2}, then the
 * stresses it started from, t^t.
 */
int or_elastic_forward(const int *n, const double *h, const double *o, int so, int nbl,
                       double dt, int nt, const double *vp, const double *vs, const double *rho,
                       double vmax_damp, int nsrc, const double *src_xyz, const double *src_wav,
                       int nrec, const double *rec_xyz, double *traces, double *state,
                       double *energy, double *hist)
{
    egrid G;
    memcpy(G.n, n, sizeof(int) * 3);
    memcpy(G.h, h, sizeof(double) * 3);
    G.r = so / 2;
    if (so < 2 || so > 16 || so % 2 || or_weights_d1_staggered(so, G.w)) return OR_EINVAL;
    const i64 N = (i64)n[0] * n[1] * n[2];
    double *F = calloc((size_t)NF * N, sizeof(double));
    double *Fold = calloc(6 * (size_t)N, sizeof(double));
    double *P = calloc((size_t)10 * N, sizeof(double));
    if (!F || !Fold || !P) {
        free(F); free(Fold); free(P);
        return OR_ENOMEM;
    }
    double *lam = P + N, *mu = P + 2 * N, *bx = P + 3 * N, *by = P + 4 * N, *bz = P + 5 * N,
           *mxy = P + 6 * N, *mxz = P + 7 * N, *myz = P + 8 * N, *dmp = P + 9 * N;
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 q = 0; q < N; q++)
            if (vp[q] > vmax) vmax = vp[q];
    }
    or_damping(n, h, nbl, vmax, dmp);
    set_params(&G, vp, vs, rho, P);
    double *vx = F + VX * N, *vy = F + VY * N, *vz = F + VZ * N;
    double *txx = F + TXX * N, *tyy = F + TYY * N, *tzz = F + TZZ * N;
    double *txy = F + TXY * N, *txz = F + TXZ * N, *tyz = F + TYZ * N;
    double ovz[3] = {o[0], o[1], o[2] + 0.5 * h[2]};
    int st = OR_OK;
    for (int t = 0; t < nt; t++) {
        /* Receivers read the current levels v^{t-1/2}, t^t. */
        if (traces) {
            for (int r = 0; r < nrec; r++) {
                double a, sxx, syy, szz;
                if ((st = interp(&G, ovz, vz, rec_xyz + 3 * r, &a))) goto done;
                if ((st = interp(&G, o, txx, rec_xyz + 3 * r, &sxx))) goto done;
                if ((st = interp(&G, o, tyy, rec_xyz + 3 * r, &syy))) goto done;
                if ((st = interp(&G, o, tzz, rec_xyz + 3 * r, &szz))) goto done;
                traces[(i64)t * nrec + r] = a;
                traces[((i64)nt + t) * nrec + r] = (sxx + syy + szz) / 3.0;
            }
        }
        if (energy) memcpy(Fold, F + TXX * N, sizeof(double) * 6 * N);
        if (hist) memcpy(hist + ((i64)t * NF + TXX) * N, F + TXX * N, sizeof(double) * 6 * N);
        /* Velocity pass. */
        vel_pass(&G, F, P, dmp, dt);
        if (hist) memcpy(hist + (i64)t * NF * N, F, sizeof(double) * 3 * N);
        /* Stress pass. */
        str_pass(&G, F, P, dmp, dt);
        /* Explosive source into the normal stresses. */
        for (int s = 0; s < nsrc; s++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(src_xyz + 3 * s, o, h, n, nodes, w);
            if (cnt < 0) { st = cnt; goto done; }
            double qv = src_wav[(i64)t * nsrc + s];
            for (int c = 0; c < cnt; c++) {
                i64 q = idx(&G, nodes[3 * c], nodes[3 * c + 1], nodes[3 * c + 2]);
                txx[q] += dt * w[c] * qv;
                tyy[q] += dt * w[c] * qv;
                tzz[q] += dt * w[c] * qv;
            }
        }
        if (energy) {
            double e = 0.0;
            for (i64 q = 0; q < N; q++) {
                e += 0.5 * (vx[q] * vx[q] / bx[q] + vy[q] * vy[q] / by[q] + vz[q] * vz[q] / bz[q]);
                /* Normal part: C^-1 = (I - lam/(3 lam + 2 mu) 1 1^T) / (2 mu). */
                const double *o6 = Fold;
                double a1 = txx[q], a2 = tyy[q], a3 = tzz[q];
                double c1 = o6[q], c2 = o6[N + q], c3 = o6[2 * N + q];
                double k = lam[q] / (3.0 * lam[q] + 2.0 * mu[q]);
                double sa = a1 + a2 + a3, sc = c1 + c2 + c3;
                e += 0.5 * ((a1 * c1 + a2 * c2 + a3 * c3) - k * sa * sc) / (2.0 * mu[q]);
                e += 0.5 * (txy[q] * o6[3 * N + q] / mxy[q] + txz[q] * o6[4 * N + q] / mxz[q] +
                            tyz[q] * o6[5 * N + q] / myz[q]);
            }
            energy[t] = e;
        }
    }
    if (state) memcpy(state, F, sizeof(double) * NF * N);
done:
    free(F);
    free(Fold);
    free(P);
    return st;
}

/*
 * Exact discrete adjoint of the linear map q -> (vz, P) traces of
 * or_elastic_forward. A step is two passes, v' = (beta v + dt b (D t)) / alpha
 * then t' = (beta t + dt C E v') / alpha (+ the source), with D the
 * divergence and E the strain operator of the staggered derivatives; with
 * every field zero outside the grid the staggered derivatives satisfy
 * (d_fwd)^T = -d_bwd, so D^T = -E and E^T = -D on these arrays, and C
 * (lambda, mu, the averaged mu) is symmetric. Backwards from zero multipliers
 * (vh, th) of the final state, for t = nt-1 .. 0:
 *   qhat^t = dt P_s (thxx + thyy + thzz)               (the source entered t^{t+1})
 *   s = th / alpha;  vh += -dt D(C s);  th = (beta/alpha) th     (stress pass)
 *   u = dt b vh / alpha;  th += -E(u);  vh = (beta/alpha) vh     (velocity pass)
 *   vh_z += P_vz^T res_vz^t;  th_ii += P^T res_P^t / 3           (receivers)
 * res[2][nt][nrec] (vz block, then P block); qhat[nt][nsrc].
 *
 * With the forward history (hist of or_elastic_forward), grad[3][N]
 * receives the gradient of J = 1/2 |traces - dobs|^2 (res = traces - dobs)
 * with respect to lambda, mu and b = 1/rho at the nodes, damping held fixed.
 * The stress pass of step t contributes, with s = th^{t+1} / alpha and e the
 * strain of v^{t+1/2},
 *   dJ/dlambda += dt tr(s) tr(e),  dJ/dmu += 2 dt sum_i s_ii e_ii  (nodes),
 *   dt s_xy e_xy (and xz, yz) at each shear point, shared 1/4 by the four
 *   nodes whose mean gives mu there;
 * the velocity pass, with vh the multiplier of v^{t+1/2} after the stress
 * pass's adjoint and D t^t the divergence of the forward stress,
 *   dt vh_a (D t^t)_a / alpha at each velocity point, shared 1/2 by the two
 *   nodes whose mean gives b there (a node beyond the grid is the nearest
 *   inside one, as in the means).
 */
static void share4(const egrid *G, double *g, i64 i, i64 j, i64 k, int a1, int a2, double c)
{
    for (int u = 0; u < 2; u++)
        for (int v = 0; v < 2; v++) {
            i64 ii = i, jj = j, kk = k;
            if (u) {
                if (a1 == 0) ii = ii + 1 < G->n[0] ? ii + 1 : G->n[0] - 1;
                if (a1 == 1) jj = jj + 1 < G->n[1] ? jj + 1 : G->n[1] - 1;
            }
            if (v) {
                if (a2 == 1) jj = jj + 1 < G->n[1] ? jj + 1 : G->n[1] - 1;
                if (a2 == 2) kk = kk + 1 < G->n[2] ? kk + 1 : G->n[2] - 1;
            }
            g[idx(G, ii, jj, kk)] += 0.25 * c;
        }
}

static void share2(const egrid *G, double *g, i64 i, i64 j, i64 k, int ax, double c)
{
    g[idx(G, i, j, k)] += 0.5 * c;
    if (ax == 0) i = i + 1 < G->n[0] ? i + 1 : G->n[0] - 1;
    if (ax == 1) j = j + 1 < G->n[1] ? j + 1 : G->n[1] - 1;
    if (ax == 2) k = k + 1 < G->n[2] ? k + 1 : G->n[2] - 1;
    g[idx(G, i, j, k)] += 0.5 * c;
}

int or_elastic_adjoint(const int *n, const double *h, const double *o, int so, int nbl,
                       double dt, int nt, const double *vp, const double *vs, const double *rho,
                       double vmax_damp, int nsrc, const double *src_xyz, int nrec,
                       const double *rec_xyz, const double *res, const double *hist,
                       double *grad, double *qhat)
{
    egrid G;
    memcpy(G.n, n, sizeof(int) * 3);
    memcpy(G.h, h, sizeof(double) * 3);
    G.r = so / 2;
    if (so < 2 || so > 16 || so % 2 || or_weights_d1_staggered(so, G.w)) return OR_EINVAL;
    const i64 N = (i64)n[0] * n[1] * n[2];
    double *F = calloc((size_t)NF * N, sizeof(double)); /* multipliers */
    double *S = calloc(6 * (size_t)N, sizeof(double));  /* C s, then u */
    double *P = calloc((size_t)10 * N, sizeof(double));
    if (!F || !S || !P) {
        free(F); free(S); free(P);
        return OR_ENOMEM;
    }
    double *lam = P + N, *mu = P + 2 * N, *bx = P + 3 * N, *by = P + 4 * N, *bz = P + 5 * N,
           *mxy = P + 6 * N, *mxz = P + 7 * N, *myz = P + 8 * N, *dmp = P + 9 * N;
    double vmax = vmax_damp;
    if (!(vmax > 0.0)) {
        vmax = 0.0;
        for (i64 q = 0; q < N; q++)
            if (vp[q] > vmax) vmax = vp[q];
    }
    or_damping(n, h, nbl, vmax, dmp);
    set_params(&G, vp, vs, rho, P);
    double *vx = F + VX * N, *vy = F + VY * N, *vz = F + VZ * N;
    double *txx = F + TXX * N, *tyy = F + TYY * N, *tzz = F + TZZ * N;
    double *txy = F + TXY * N, *txz = F + TXZ * N, *tyz = F + TYZ * N;
    double *sxx = S, *syy = S + N, *szz = S + 2 * N, *sxy = S + 3 * N, *sxz = S + 4 * N,
           *syz = S + 5 * N;
    double ovz[3] = {o[0], o[1], o[2] + 0.5 * h[2]};
    int st = OR_OK;
    if (qhat) memset(qhat, 0, sizeof(double) * (size_t)nt * nsrc);
    if (grad && !hist) {
        st = OR_EINVAL;
        goto done;
    }
    if (grad) memset(grad, 0, sizeof(double) * 3 * N);
    for (int t = nt - 1; t >= 0; t--) {
        if (grad) {
            /* Stress-pass terms: s = th^{t+1} / alpha against e(v^{t+1/2}). */
            const double *hv = hist + (i64)t * NF * N;
            const double *hvx = hv, *hvy = hv + N, *hvz = hv + 2 * N;
            double *gl = grad, *gm = grad + N;
            for (i64 i = 0; i < n[0]; i++)
                for (i64 j = 0; j < n[1]; j++)
                    for (i64 k = 0; k < n[2]; k++) {
                        i64 q = idx(&G, i, j, k);
                        const double al = 1.0 + dmp[q] * dt / 2.0;
                        const double exx = dst(&G, hvx, i, j, k, 0, 0),
                                     eyy = dst(&G, hvy, i, j, k, 1, 0),
                                     ezz = dst(&G, hvz, i, j, k, 2, 0);
                        const double a = txx[q] / al, bb = tyy[q] / al, c = tzz[q] / al;
                        gl[q] += dt * (a + bb + c) * (exx + eyy + ezz);
                        gm[q] += 2.0 * dt * (a * exx + bb * eyy + c * ezz);
                        const double gxy = dst(&G, hvx, i, j, k, 1, 1) + dst(&G, hvy, i, j, k, 0, 1);
                        const double gxz = dst(&G, hvx, i, j, k, 2, 1) + dst(&G, hvz, i, j, k, 0, 1);
                        const double gyz = dst(&G, hvy, i, j, k, 2, 1) + dst(&G, hvz, i, j, k, 1, 1);
                        share4(&G, gm, i, j, k, 0, 1, dt * txy[q] / al * gxy);
                        share4(&G, gm, i, j, k, 0, 2, dt * txz[q] / al * gxz);
                        share4(&G, gm, i, j, k, 1, 2, dt * tyz[q] / al * gyz);
                    }
        }
        for (int s = 0; qhat && s < nsrc; s++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(src_xyz + 3 * s, o, h, n, nodes, w);
            if (cnt < 0) { st = cnt; goto done; }
            double acc = 0.0;
            for (int c = 0; c < cnt; c++) {
                i64 q = idx(&G, nodes[3 * c], nodes[3 * c + 1], nodes[3 * c + 2]);
                acc += dt * w[c] * (txx[q] + tyy[q] + tzz[q]);
            }
            qhat[(i64)t * nsrc + s] = acc;
        }
        /* Adjoint of the stress pass. */
        for (i64 q = 0; q < N; q++) {
            const double al = 1.0 + dmp[q] * dt / 2.0, be = 1.0 - dmp[q] * dt / 2.0;
            const double a = txx[q] / al, bb = tyy[q] / al, c = tzz[q] / al;
            const double tr = a + bb + c;
            sxx[q] = lam[q] * tr + 2.0 * mu[q] * a;
            syy[q] = lam[q] * tr + 2.0 * mu[q] * bb;
            szz[q] = lam[q] * tr + 2.0 * mu[q] * c;
            sxy[q] = mxy[q] * txy[q] / al;
            sxz[q] = mxz[q] * txz[q] / al;
            syz[q] = myz[q] * tyz[q] / al;
            for (int f = TXX; f <= TYZ; f++) F[f * N + q] *= be / al;
        }
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n[0]; i++)
            for (i64 j = 0; j < n[1]; j++)
                for (i64 k = 0; k < n[2]; k++) {
                    i64 q = idx(&G, i, j, k);
                    vx[q] -= dt * (dst(&G, sxx, i, j, k, 0, 1) + dst(&G, sxy, i, j, k, 1, 0) +
                                   dst(&G, sxz, i, j, k, 2, 0));
                    vy[q] -= dt * (dst(&G, sxy, i, j, k, 0, 0) + dst(&G, syy, i, j, k, 1, 1) +
                                   dst(&G, syz, i, j, k, 2, 0));
                    vz[q] -= dt * (dst(&G, sxz, i, j, k, 0, 0) + dst(&G, syz, i, j, k, 1, 0) +
                                   dst(&G, szz, i, j, k, 2, 1));
                }
        if (grad) {
            /* Velocity-pass terms: vh (now complete) against D t^t. */
            const double *ht = hist + ((i64)t * NF + TXX) * N;
            const double *hxx = ht, *hyy = ht + N, *hzz = ht + 2 * N, *hxy = ht + 3 * N,
                         *hxz = ht + 4 * N, *hyz = ht + 5 * N;
            double *gb = grad + 2 * N;
            for (i64 i = 0; i < n[0]; i++)
                for (i64 j = 0; j < n[1]; j++)
                    for (i64 k = 0; k < n[2]; k++) {
                        i64 q = idx(&G, i, j, k);
                        const double al = 1.0 + dmp[q] * dt / 2.0;
                        const double fx = dst(&G, hxx, i, j, k, 0, 1) + dst(&G, hxy, i, j, k, 1, 0) +
                                          dst(&G, hxz, i, j, k, 2, 0);
                        const double fy = dst(&G, hxy, i, j, k, 0, 0) + dst(&G, hyy, i, j, k, 1, 1) +
                                          dst(&G, hyz, i, j, k, 2, 0);
                        const double fz = dst(&G, hxz, i, j, k, 0, 0) + dst(&G, hyz, i, j, k, 1, 0) +
                                          dst(&G, hzz, i, j, k, 2, 1);
                        share2(&G, gb, i, j, k, 0, dt * vx[q] / al * fx);
                        share2(&G, gb, i, j, k, 1, dt * vy[q] / al * fy);
                        share2(&G, gb, i, j, k, 2, dt * vz[q] / al * fz);
                    }
        }
        /* Adjoint of the velocity pass: u = dt b vh / alpha into S[0..2]. */
        for (i64 q = 0; q < N; q++) {
            const double al = 1.0 + dmp[q] * dt / 2.0, be = 1.0 - dmp[q] * dt / 2.0;
            sxx[q] = dt * bx[q] * vx[q] / al;
            syy[q] = dt * by[q] * vy[q] / al;
            szz[q] = dt * bz[q] * vz[q] / al;
            vx[q] *= be / al;
            vy[q] *= be / al;
            vz[q] *= be / al;
        }
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n[0]; i++)
            for (i64 j = 0; j < n[1]; j++)
                for (i64 k = 0; k < n[2]; k++) {
                    i64 q = idx(&G, i, j, k);
                    txx[q] -= dst(&G, sxx, i, j, k, 0, 0);
                    tyy[q] -= dst(&G, syy, i, j, k, 1, 0);
                    tzz[q] -= dst(&G, szz, i, j, k, 2, 0);
                    txy[q] -= dst(&G, sxx, i, j, k, 1, 1) + dst(&G, syy, i, j, k, 0, 1);
                    txz[q] -= dst(&G, sxx, i, j, k, 2, 1) + dst(&G, szz, i, j, k, 0, 1);
                    tyz[q] -= dst(&G, syy, i, j, k, 2, 1) + dst(&G, szz, i, j, k, 1, 1);
                }
        /* Receivers of step t (they read v^{t-1/2} and t^t). */
        for (int r = 0; r < nrec; r++) {
            int nodes[24];
            double w[8];
            int cnt = or_trilinear(rec_xyz + 3 * r, ovz, h, n, nodes, w);
            if (cnt < 0) { st = cnt; goto done; }
            const double rv = res[(i64)t * nrec + r];
            for (int c = 0; c < cnt; c++)
                vz[idx(&G, nodes[3 * c], nodes[3 * c + 1], nodes[3 * c + 2])] += w[c] * rv;
            cnt = or_trilinear(rec_xyz + 3 * r, o, h, n, nodes, w);
            if (cnt < 0) { st = cnt; goto done; }
            const double rp = res[((i64)nt + t) * nrec + r] / 3.0;
            for (int c = 0; c < cnt; c++) {
                i64 q = idx(&G, nodes[3 * c], nodes[3 * c + 1], nodes[3 * c + 2]);
                txx[q] += w[c] * rp;
                tyy[q] += w[c] * rp;
                tzz[q] += w[c] * rp;
            }
        }
    }
done:
    free(F);
    free(S);
    free(P);
    return st;
}

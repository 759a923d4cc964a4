// Kernel arguments of the TTI step kernels (tti.hip).
#pragma once

#include "tb_internal.h"

namespace tbw {

struct TtiParams {
    const float *p, *r;  // current levels p^n, r^n        [nx][ny][nzp]
    float *vp, *vr;      // p^n - p^{n-1}, r^n - r^{n-1}; updated in place
    float *pn, *rn;      // receive p^{n+1}, r^{n+1}
    float *qp, *qr;      // rotated gradients (scratch)
    const float *ax, *ay, *az;  // symmetry axis per node
    const float *e1, *sd;       // 1 + 2 eps, sqrt(1 + 2 min(delta, eps))
    const float *c;             // dt^2 vp^2
    const float *dx, *dy, *dz;  // damping per axis
    float hdt;                  // dt / 2
    float w1[6];                // centred first derivative, unit spacing
    float w2[7];                // centred second derivative, unit spacing
    float ih[3], ih2[3];        // 1/h and 1/h^2 per axis
    int nx, ny, nz, nzp;
    // Adjoint step only: lambda^{k+1} (lp, lr) and the mixed fields
    // z = (c/alpha) D lambda^{k+1} (zp, zr), which p and r then point to.
    const float *lp, *lr;
    float *zp, *zr;
    // Planes [xlo, xhi) a launch computes (xhi = 0: all of x), and where the
    // forward update writes the new velocities (NULL: in place over vp, vr).
    // Temporally blocked passes compute shrinking x ranges into separate
    // buffers; every buffer is addressed with the global (x, y, z) offsets.
    int xlo, xhi;
    float *vpo, *vro;
    // XCD-aware block order of the forward launches (0: linear): runs of
    // 8 * band blocks, of which XCD k takes the k-th contiguous band.
    int band;
    // Streaming launches: planes per workgroup and chunks per tile (set by
    // the launch), and the device's compute units (set with the model).
    int chunk, nchunks;
    int ncu;
};

// One step: rotated gradients, coupled update (velocity form), injection of
// inc[npts] at soff into both fields, gather of p^{n+1} into rec_row[nrid] at
// roff. The update covers planes [P.xlo, P.xhi), the rotated gradients that
// range widened by the radius, and injection every point of the update's
// range; receivers are gathered at the points of planes [rlo, rhi) only.
tb_status launch_tti_step(const TtiParams &P, int r, const float *inc, const long long *soff,
                          int npts, float *rec_row, const long long *roff, int nrid, int rlo,
                          int rhi, hipStream_t st);

// One step of the adjoint of q -> d, backwards: lambda^{k+1} in (P.lp, P.lr),
// psi^{k+1} = lambda^{k+1} - lambda^{k+2} in (P.vp, P.vr) (updated in place
// to psi^k), lambda^k into (P.pn, P.rn). First src_row[npts] receives
// c (lambda_p + lambda_r)^{k+1} / alpha at the source points (soff, alpha per
// point), then z = (c/alpha) D lambda^{k+1} goes to (P.zp, P.zr), and
//   psi^k = H z + (beta/alpha) psi^{k+1} + (P_r^T res^k, 0),
//   lambda^k = lambda^{k+1} + psi^k,
// with H = diag(L - Hz, Hz) and res^k decomposed at the receiver points as
// inc[nrid] (added at roff).
// Imaging term of the gradient for a forward level w = (P.p, P.r) against
// the multiplier lambda^{k+1} = (P.lp, P.lr): the rotated gradients of w go
// to (P.qp, P.qr), then g += sum_f y_f c (A w)_f with y = (c/alpha) lambda
// (g in FP64, padded layout).
tb_status launch_tti_image(const TtiParams &P, int r, double *g, hipStream_t st);
// gs[i] += row[i] alpha[i] inc[i] at the source points.
tb_status launch_tti_image_sparse(const float *row, const double *alpha, const float *inc,
                                  int npts, double *gs, hipStream_t st);

tb_status launch_tti_adjoint_step(const TtiParams &P, int r, const float *inc,
                                  const long long *roff, int nrid, float *src_row,
                                  const long long *soff, const double *src_alpha, int npts,
                                  hipStream_t st);

}  // namespace tbw

// Kernel arguments of the elastic step kernels (elastic.hip).
#pragma once

#include "tb_internal.h"

namespace tbw {

struct ElParams {
    float *v[3];              // vx, vy, vz                     [nx][ny][nzp]
    float *t[6];              // txx, tyy, tzz, txy, txz, tyz
    const float *bq[3];       // dt * b at the vx, vy, vz points
    const float *lam, *mu;    // dt * lambda, dt * mu at the nodes
    const float *ms[3];       // dt * mu at the txy, txz, tyz points
    const float *dx, *dy, *dz;  // damping per axis
    float hdt;                // dt / 2
    float w[6];               // staggered first derivative, unit spacing
    float ih[3];              // 1/h per axis
    int nx, ny, nz, nzp;
    // Planes [xlo, xhi) a launch computes (xhi = 0: all of x), and where the
    // forward passes write (NULL: in place over v, t). Temporally blocked
    // passes compute shrinking x ranges into separate buffers; every buffer
    // is addressed with the global (x, y, z) offsets.
    int xlo, xhi;
    float *vo[3];
    float *to[6];
    // XCD-aware block order of the forward launches (0: linear): runs of
    // 8 * band blocks, of which XCD k takes the k-th contiguous band.
    int band;
    // Streaming launches: planes per workgroup and chunks per tile (set by
    // the launch), and the device's compute units (set with the model).
    int chunk, nchunks;
    int ncu;
};

// Six scratch fields of the adjoint step (also used to pass a forward
// level: v in f[0..2], or t in f[0..5]).
struct ElScratch {
    float *f[6];
};

// FP64 gradient accumulators (padded layout): node terms of lambda and mu,
// per-shear-point and per-velocity-point terms before their spread onto the
// nodes.
struct ElGradAcc {
    double *lam, *mu;
    double *sh[3];  // xy, xz, yz
    double *bv[3];  // x, y, z
};

// One backward step of the gradient: the stress-pass imaging against the
// forward v^{t+1/2} (fv), the stress-pass adjoint, the velocity-pass imaging
// against the forward t^t (ft), the velocity-pass adjoint, the receivers.
tb_status launch_elastic_gradient_step(const ElParams &P, const ElScratch &S,
                                       const ElScratch &fv, const ElScratch &ft,
                                       const ElGradAcc &G, int r, const float *inc_p,
                                       const long long *roff, int nrid, const float *inc_v,
                                       const long long *roff2, int nrid2, double dt,
                                       hipStream_t st);
// Spreads the element terms onto the nodes and writes out[3][nx][ny][nz] =
// (dJ/dlambda, dJ/dmu, dJ/db).
tb_status launch_elastic_grad_finish(const ElParams &P, const ElGradAcc &G, float *out,
                                     hipStream_t st);

// One step of the adjoint of q -> (vz, P), backwards: multipliers of the
// velocities in P.v and of the stresses in P.t (in place). First src_row
// receives dt (thxx + thyy + thzz) / alpha at the source points (soff, alpha
// per point); then the stress-pass adjoint (S = C th / alpha, vh -= div S,
// th *= beta/alpha), the velocity-pass adjoint (S = dt b vh / alpha,
// th -= strain S, vh *= beta/alpha), and the receivers of the step (th_ii +=
// inc_p / 3 at roff, vh_z += inc_v at roff2).
tb_status launch_elastic_adjoint_step(const ElParams &P, const ElScratch &S, int r,
                                      const float *inc_p, const long long *roff, int nrid,
                                      const float *inc_v, const long long *roff2, int nrid2,
                                      float *src_row, const long long *soff,
                                      const double *src_alpha, double dt, int npts,
                                      hipStream_t st);

// One step: velocity and stress passes (in place, or into P.vo / P.to),
// injection of inc[npts] at soff into the three normal stresses, gather of P
// into row_p[nrid] at roff and of vz into row_v[nrid2] at roff2. The stress
// pass and the injection cover planes [P.xlo, P.xhi), the velocity pass that
// range widened by the radius; receivers are gathered at the points of
// planes [rlo, rhi) only.
tb_status launch_elastic_step(const ElParams &P, int r, const float *inc, const long long *soff,
                              int npts, float *row_p, const long long *roff, int nrid,
                              float *row_v, const long long *roff2, int nrid2, int rlo, int rhi,
                              hipStream_t st);

}  // namespace tbw

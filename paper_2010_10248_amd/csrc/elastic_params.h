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
};

// One step: velocity and stress passes (in place), injection of inc[npts] at
// soff into the three normal stresses, gather of P into row_p[nrid] at roff
// and of vz into row_v[nrid2] at roff2.
tb_status launch_elastic_step(const ElParams &P, int r, const float *inc, const long long *soff,
                              int npts, float *row_p, const long long *roff, int nrid,
                              float *row_v, const long long *roff2, int nrid2, hipStream_t st);

}  // namespace tbw

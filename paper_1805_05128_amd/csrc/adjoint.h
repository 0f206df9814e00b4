// Launchers of the adjoint's piston handling (k_adjoint.hip): the gather split into a pass
// without the wall and a mirror-only pass over the wall band; for the Euler step's VJP, the
// step's reflections found from the gathers' own rate sums, then a correction gather over the
// band.
#pragma once

#include "csph_internal.h"

namespace csph {

// The two gathers of a step VJP with the piston.  First pass (svy set): the gathers take the
// next state's cotangent as given and leave each particle's y-momentum rate sum, from which
// k_wall_flags tests the step's reflection, y + dt (v_y + dt R_vy) < yw1 (kernels' y), and
// raises reach (order_enc) to max(y, 2 y_w - y) over the flagged particles.  Correction pass
// (band set): the gathers of the cotangent change the reflection's transpose makes,
// accumulated; only workgroups holding a particle with y within the support of the decoded
// reach walk their stencils (no other particle has a partner whose change is not zero), the
// rest write zero EOS-parameter partial sums and return.
struct WallPass {
    double *svy;                     // first pass: the y-momentum rate sums S_vy (cell order)
    const unsigned long long *band;  // correction pass: the reach of the flagged particles
};

// The gather with the piston in two launches: one without the wall for every particle, then
// the mirror walks for the workgroups holding wall-band particles, added to its outputs.
// Rate cotangents a_in (rates VJP), or the next state's cotangent gnext (step VJP).
hipError_t launch_vjp_wall(int64_t n, const int32_t *perm, const int32_t *cs, const GridDev &g,
                           const PairConst &pc, const EosDev &eos, const Ws &w,
                           double *const sorted[9], const int32_t *mat_sorted,
                           const double *const a_in[5], double *const gout[8],
                           const double *const gnext[8], double dt, int accumulate,
                           double *g_eos, const double *d_sorted, double yw, double vw,
                           const WallPass &wp, hipStream_t st);

// The step's reflections from the first pass's rate sums: flag (input order) and reach.
hipError_t launch_wall_flags(int64_t n, const int32_t *perm, double *const sorted[9],
                             const double *svy, double dt, double yw1, double yw, int32_t *flag,
                             unsigned long long *reach, hipStream_t st);

// The cotangent change a reflection makes to y and v_y: d_y = -2 g_y, d_vy = -2 g_vy - 2 v_w g_E
// (input order), formed for every particle before the first pass (which may overwrite g when
// the output aliases it) ...
hipError_t launch_reflect_delta(int64_t n, const double *gy, const double *gvy, const double *gE,
                                double vw, double *dy, double *dvy, hipStream_t st);
// ... and kept after it for the flagged particles only (zero elsewhere).
hipError_t launch_keep_flagged(int64_t n, const int32_t *flag, double *dy, double *dvy,
                               hipStream_t st);

}  // namespace csph

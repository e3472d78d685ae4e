// Free-fall bookkeeping shared by the 2D and axisymmetric flow steps
// (Section 2.1: non-inertial frame, conservation of mass). Host only; no HIP
// types, so the host-compiled unit that defines it can include it.
#pragma once

#include "../../include/ibproj.h"

namespace ib {

struct FreeFall {
    double com0 = 0.0;       // vertical centroid of the first step's markers
    double com_prev = 0.0;   // that of the previous step's markers
    double vol0 = 0.0;       // enclosed area / volume of the first step
    long nstep = 0;          // steps taken since the reset
    int have = 0;
};

// Before a step on the incoming markers X (n x 2, host): fills stats->com,
// stats->measure and stats->frame_a (fp->frame: a = -c1 (COM_n - COM_0)/dt -
// c2 (COM_n - COM_{n-1})/dt, else 0), and *mass_target with the first step's
// measure (fp->mass_target when positive) when this step's relocated markers
// take the mass correction (NULL otherwise). Does nothing but clear the stats when neither is on.
// With nt > 0, X is a closed mesh (n vertices x 3, triangles T, host) and the
// measure is its volume and the y of its centroid.
int freefall_begin(FreeFall* s, const ib_flow_params* fp, int n, const double* X, double axis_x,
                   double dt, ib_flow_stats* stats, const double** mass_target, int nt = 0,
                   const int* T = nullptr);

}  // namespace ib

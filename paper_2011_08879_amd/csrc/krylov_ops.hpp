// Reduction-finishing operations shared by the CGS kernels and the fused
// products (one thread applies the recurrence's scalar step to the totals).
#pragma once

#include <cmath>

#include "solver_state.hpp"

namespace gko {

// alpha = rho / (t.rhat)
struct cgs_alpha_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->aux = o[0];
        if (!(fabs(o[0]) >= 1e-300)) sc->done = kBreakdown;
        else sc->alpha = sc->rho / o[0];
    }
};

}  // namespace gko

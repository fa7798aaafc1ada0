// Device-resident scalars of the Krylov solvers.  Every step kernel reads them
// and the last block of each reduction writes them, so an iteration needs no
// host round trip; the host polls `done` every few iterations.
#pragma once

#include <stdint.h>

namespace gko {

enum solver_flag : int32_t {
    kRunning = 0,
    kConverged = 1,
    kNotSpd = 2,
    kBreakdown = 3,
    kMaxIter = 4,
};

struct krylov_scalars {
    double rho;       // CG: r.z        BiCGSTAB: rhat.r
    double rho_old;   // BiCGSTAB
    double alpha;
    double beta;
    double omega;     // BiCGSTAB
    double rr;        // r.r of the latest residual
    double bb;        // b.b
    double stop2;     // rr threshold: tol^2 * bb
    double aux;       // last denominator (p.q, rhat.v or t.t), for diagnostics
    int32_t iter;     // completed iterations
    int32_t maxit;    // iteration cap
    int32_t done;     // solver_flag
    int32_t half;     // BiCGSTAB: converged at the half step, x += alpha p pending
};

}  // namespace gko

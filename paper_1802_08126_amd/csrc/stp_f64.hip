// Typed solver instantiation: storage double, compute double.
#define STP_SOLVER_TU 1
#include "stp_solver.h"

namespace stpx {
SolverBase* make_solver_f64(stp_ctx* c) { return new Solver<double, double>(c); }
}  // namespace stpx

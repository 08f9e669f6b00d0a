// Typed solver instantiation: storage float, compute float.
#define STP_SOLVER_TU 1
#include "stp_solver.h"

namespace stpx {
SolverBase* make_solver_f32(stp_ctx* c) { return new Solver<float, float>(c); }
}  // namespace stpx

// Typed solver instantiation: storage bf16, compute float.
#define STP_SOLVER_TU 1
#include "stp_solver.h"

namespace stpx {
SolverBase* make_solver_bf16(stp_ctx* c) { return new Solver<bf16, float>(c); }
}  // namespace stpx

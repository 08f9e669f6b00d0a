"""MI355X-native space-time parallel solver for linear parabolic equations.

Implements the inexact Uzawa iteration on the symmetric saddle-point form of
implicit Euler with the DST-in-time Schur complement preconditioner
(Neumueller & Smears, "Time-parallel iterative solvers for parabolic evolution
equations", Sections 2-4) as hand-written HIP kernels for gfx950 behind the C
ABI of include/stp.h.  This package is the ctypes binding of that library.
"""
from .binding import (  # noqa: F401
    STP_OP_B,
    STP_OP_SADDLE,
    STP_PC_A,
    STP_PC_H,
    STP_OK,
    STP_EINVAL,
    STP_ENOMEM,
    STP_EDEVICE,
    STP_ENOTCONV,
    STP_EDIVERGED,
    STP_EUNSUPPORTED,
    BatchSolver,
    SpaceTimeSolver,
    StpError,
    from_problem,
    problem_dict,
    lib_path,
    load,
    stp_apply_operator,
    stp_apply_precond,
    stp_autotune,
    stp_batch_size,
    stp_create,
    stp_create_batch,
    stp_destroy,
    stp_device_bytes_allocated,
    stp_gmres_solve,
    stp_gmres_workspace_bytes,
    stp_omega_info,
    stp_set_omega,
    stp_set_stop,
    stats_dict,
    stp_schedule_string,
    stp_timing_enable,
    stp_timing_report,
    stp_uzawa_solve,
    stp_uzawa_solve_batch,
    stp_workspace_bytes,
    stp_workspace_bytes_batch,
)

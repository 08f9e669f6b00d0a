// Internal host-side declarations shared by the translation units of
// libstp: problem and launch-table structures, the context, the timing
// hooks and the launch macros, and the interface of the typed solvers
// (one translation unit per precision, compiled in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "stp.h"
#include "stp_fem.h"
#include "stp_kernels.h"
#include "stp_tiles.h"
#include "stp_pencil.h"

struct stp_ctx;

namespace stpx {
using namespace stp;

// records the detail message of the calling thread and returns s
stp_status fail(stp_status s, const char* fmt, ...);
}  // namespace stpx

void kt_end(stp_ctx* c);

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(STP_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),     \
                  __FILE__, __LINE__);                                                    \
  } while (0)

#define LAUNCH_CHECK()                                                                    \
  do {                                                                                    \
    kt_end(&*c);                                                                          \
    hipError_t _e = hipGetLastError();                                                    \
    if (_e != hipSuccess)                                                                 \
      return fail(STP_EDEVICE, "kernel launch failed: %s (%s:%d)", hipGetErrorString(_e), \
                  __FILE__, __LINE__);                                                    \
  } while (0)

namespace stpx {


// finite-element stencils of one level (M and A, scaled to the Galerkin level)
struct FemLevelW {
  double m[27];
  double a[27];
};

struct Level {
  int n;
  double h;
  Geom g;
  void* fr = nullptr;   // finite elements: two TS iterates of the level's Jacobi sweeps
  void* fr2 = nullptr;
  double* kraw;    // unscaled nodal fields (float64), R x nnodes (level 0: the caller's)
  void* kscaled;   // TC fields scaled by 0.5/h^2
  void* b;         // TS right-hand side of the level (levels >= 1)
  void* e;         // TS correction produced on the level (levels >= 1)
  // register-pencil down-sweep fields of the A (0) and H (1) families: the fixed
  // field and its face sums at the interior nodes (TC), or null
  bool pen[2] = {false, false};   // set in the planning dry run too (null pk, pd there)
  void* pk[2] = {nullptr, nullptr};
  void* pd[2] = {nullptr, nullptr};
};

// 3-D multigrid levels l whose down-sweep runs as register pencils: the
// level's family-fam operator is a fixed field times a slab scalar (always for
// the H family, for the A family when the coefficient has rank 1), the coarse
// level is wide enough to fill the pencils' lanes, and a slab of the fine level
// addresses below 2 GiB (32-bit buffer offsets).
inline bool pencil_level(int dim, int spatial, bool fem, int R, int nf, int nc, size_t tsb, size_t tcb, int fam) {
  if (dim != 3 || spatial != STP_SPATIAL_MG || fem) return false;
  if (fam == 0 && R != 1) return false;
  if (nc < kPencilMinNc) return false;
  const double bytes = double(nf) * nf * nf * double(std::max(tsb, tcb));
  return bytes < double(1u << 31) - 65536.0;
}

struct Bump {
  char* base = nullptr;
  size_t off = 0;
  bool dry = true;
  void* take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    void* p = dry ? nullptr : base + off;
    off += bytes;
    return p;
  }
};

inline size_t ts_bytes(int prec) { return prec == STP_PREC_F64 ? 8 : (prec == STP_PREC_F32 ? 4 : 2); }
inline size_t tc_bytes(int prec) { return prec == STP_PREC_F64 ? 8 : 4; }

inline long ipow(long a, int d) {
  long r = 1;
  for (int i = 0; i < d; ++i) r *= a;
  return r;
}

inline dim3 grid_pts(long npts, int S) {
  const long bx = (npts + kBlock - 1) / kBlock;
  const int gy = std::min(S, 65535);
  const int gz = (S + 65534) / 65535;
  return dim3(unsigned(bx), unsigned(gy), unsigned(gz));
}

enum { TP_FFT2 = 0, TP_STOCKHAM = 1, TP_DENSE = 2, TP_BLUESTEIN = 3, TP_FOUR = 4 };

constexpr int kNormBlocks = 1024;     // blocks of the finite-element residual-norm pass after a solve
constexpr int kBlueKey = 1 << 20;        // site key of a Bluestein group: kBlueKey + M
constexpr int kBlueMaxN = 2048;          // Bluestein for step counts up to this (M <= 4096)
constexpr size_t kMaxLds = 160 * 1024;   // LDS of one compute unit
constexpr int kFourMaxN = 1 << 20;       // four-step FFT for powers of two above 4096 up to this

// four-step FFT: LDS of a pass (FFT length N1 >= N2, C columns) and default columns
inline size_t four_lds(int N, int C, size_t tcb) {
  const int N1 = four_n1(N);
  return (size_t(2) * N1 * C + size_t(2) * N1) * tcb;
}
inline int four_cols(int N) { return std::max(1, std::min(16, 4096 / four_n1(N))); }
inline size_t stockham_lds(int N, int C, size_t tcb);
// powers of two the in-LDS Stockham FFT cannot take (N > 4096, or one column
// too large for the LDS) run as four-step FFTs
inline bool four_step_n(int N, size_t tcb) {
  const bool pow2 = N >= 1 && (N & (N - 1)) == 0;
  return pow2 && N >= 512 && N <= kFourMaxN && (N > 4096 || stockham_lds(N, 1, tcb) > kMaxLds);
}

// Bluestein FFT length: the smallest power of two >= 2N - 1
inline int bluestein_M(int N) {
  int M = 1;
  while (M < 2 * N - 1) M *= 2;
  return M;
}
inline size_t bluestein_lds(int M, int C, size_t tcb) { return (size_t(2) * M * C + size_t(2) * M) * tcb; }
inline int bluestein_cols(int M, size_t tcb) {
  int C = 16;
  while (C > 1 && (M * C > 4096 || bluestein_lds(M, C, tcb) > kMaxLds)) C /= 2;
  return C;
}

// Default transform path for N: two-step register FFT (4 <= N <= 256, power
// of two), Stockham LDS FFT (other powers of two up to 4096), Bluestein
// (other N from 17 to 2048), dense otherwise.
inline void transform_path(int N, size_t tcb, int& path, int& C, size_t& lds) {
  C = 0;
  lds = 0;
  const bool pow2 = N >= 1 && (N & (N - 1)) == 0;
  if (pow2 && N >= 4 && N <= 256) {
    path = TP_FFT2;
    return;
  }
  if (pow2 && N <= 4096) {
    C = std::max(1, std::min(16, 4096 / N));
    lds = (size_t(2) * N * C + size_t(4) * N) * tcb;
    if (lds <= kMaxLds) {
      path = TP_STOCKHAM;
      return;
    }
  }
  if (four_step_n(N, tcb)) {
    C = four_cols(N);
    lds = four_lds(N, C, tcb);
    path = TP_FOUR;
    return;
  }
  if (!pow2 && N > 16 && N <= kBlueMaxN) {
    const int M = bluestein_M(N);
    C = bluestein_cols(M, tcb);
    lds = bluestein_lds(M, C, tcb);
    path = TP_BLUESTEIN;
    return;
  }
  C = 0;
  lds = 0;
  path = TP_DENSE;
}

// site key of a step count: N (powers of two up to 4096), the Bluestein group
// kBlueKey + M (other N up to kBlueMaxN), or -1 (the dense group)
inline int transform_key(int N) {
  if (N >= 1 && (N & (N - 1)) == 0 && N <= kFourMaxN) return N;
  if (N <= kBlueMaxN) return kBlueKey + bluestein_M(N);
  return -1;
}

inline bool is_pow2(int N) { return N >= 1 && (N & (N - 1)) == 0; }

// Stockham LDS bytes for N points and C columns per block
inline size_t stockham_lds(int N, int C, size_t tcb) { return (size_t(2) * N * C + size_t(4) * N) * tcb; }

// Schedule knobs of the tile launches.  Each knob scales the slabs per
// block of every job of its launch sites by 2^e relative to the heuristic.
enum Knob {
  KN_R0 = 0,            // residual r_p
  KN_R1,                // residual r_u (and the stop-test partials)
  KN_MID,               // middle reference operator of the H-blocks
  KN_UPA0,              // finest up-sweep of the A-tilde cycle (float64 accumulation)
  KN_DOWN0,             // down-sweep into level l + 1 (all three cycles)
  KN_UP0 = KN_DOWN0 + STP_MAX_LEVELS,   // up-sweep on level l, stored output
  KN_FUSE = KN_UP0 + STP_MAX_LEVELS,    // threads per block of the fused coarse levels: 256 << e
  KN_COUNT
};

struct TransformChoice {
  int path;
  int C;      // Stockham columns per block
};

struct Schedule {
  int e[KN_COUNT];
  std::map<int, TransformChoice> tpath;   // per power-of-two step count
  Schedule() {
    std::fill(e, e + KN_COUNT, 0);
    e[KN_FUSE] = 2;   // 1024 threads: the fused kernel has one block per slab
  }
};

struct Problem {
  int dim = 0, n = 0, N = 0, R = 0;
  double tau = 0;               // reference step of eq. (2.2) (the step when uniform)
  std::vector<double> taus;     // N step lengths tau_n
  const double* F = nullptr;
  const double* u0 = nullptr;
  const double* fields = nullptr;
  std::vector<double> tcoef;   // R x N
  std::vector<double> abar;    // R
  std::vector<Level> lv;
  Geom g0{};
  int tpath = TP_DENSE;         // default transform path (the tuner may choose another)
  long resid_tiles = 0;
  int fuse_top = 0;             // first multigrid level solved by the fused coarse kernel
  long npart = 0;               // residual partials (one per block of the a3 residual launch)
  double omega = 0.8;           // damping of the u-update (eq. (3.1))
  bool omega_auto = false;      // omega estimated at setup
  double est_lmin = 0, est_lmax = 0, est_rho = 0;   // estimates behind an automatic omega
  long nfnorm = 0;              // partials of the setup reduction of ||f||
  // device memory
  DevState* state = nullptr;
  double* partial = nullptr;
  double* nrm = nullptr;        // partials of the returned pair's residual norms (two rows)
  void* njob = nullptr;         // device job of the residual-norm pass (ResidJob)
  double* kap64 = nullptr;      // finest-level scaled fields, float64
  double* cA64 = nullptr;       // N x kMaxRank: tau_n * tcoef
  double* taus64 = nullptr;     // N step lengths
  void* cA = nullptr;           // TC, N x kMaxRank
  void* sigH = nullptr;         // TC, N: mu_k
  void* cH = nullptr;           // TC, N x kMaxRank: tau * abar
  void* cMid = nullptr;         // TC, kMaxRank: (2/N) tau abar
  void* sinT = nullptr;         // TC, N x N (dense path)
  void* sinM = nullptr;
  void* tw = nullptr;           // TC, 2N (Bluestein problems: w_M, 2M)
  void* tw4 = nullptr;          // TC, 2N
  int blM = 0;                  // Bluestein FFT length (0: not a Bluestein step count)
  void* chirp = nullptr;        // TC, 2N
  void* bhat = nullptr;         // TC, 2M
  void* fs = nullptr;           // TC, 2 x N x n^d: four-step FFT scratch (powers of two > 4096)
  void* W1 = nullptr;           // TS, N x n^d
  void* W2 = nullptr;
  void* Xnu = nullptr;          // TS, N x n^d: correction of one cycle when nu_A or nu_H > 1
  void* tri = nullptr;          // TC scratch of exact 1-D solves, 2 x N x n
  double fnorm = 0;
  // finite elements: stencils per level and the binding of the current solve
  std::vector<FemLevelW> fw;
  FemBind* fbind = nullptr;
};

// operator family of the V-cycles: 0 A-tilde (tau_n A_n), 1 the H-blocks, 2 the middle operator
inline LevelOp family_op(const Problem& q, int l, int fam) {
  LevelOp L;
  L.kap = q.lv[l].kscaled;
  L.R = q.R;
  L.S = q.N;
  if (fam == 0) {          // A family: tau_n A_n (rank 1: the field times tau a_0[n])
    L.sig = nullptr;
    L.c = q.cA;
    L.cmode = q.R == 1 ? CM_SCALE : CM_SLAB;
  } else if (fam == 1) {   // H family: mu_k I + tau A_ref (the same coefficient for every k)
    L.sig = q.sigH;
    L.c = q.cH;
    L.cmode = CM_UNIFORM;
  } else {                 // middle: (2/N) tau A_ref
    L.sig = nullptr;
    L.c = q.cMid;
    L.cmode = CM_UNIFORM;
  }
  return L;
}

template <typename J>
struct Site {
  std::vector<J> jobs;
  J* dev = nullptr;
  long blocks = 0;
  int key = 0;     // transform sites: N (-1: the dense group of other step counts)
  size_t shmem = 0;               // fused multigrid sites: dynamic LDS of the launch
  int threads = 256;              // fused multigrid sites: threads per block
  bool fixed = true;              // tile sites: every job's coefficient is a fixed field times a slab scalar
  bool anyfix = false;            // tile sites: at least one job's coefficient is a fixed field
  int epi = 0;
  int path = TP_DENSE, C = 0;   // transform sites: path and Stockham columns
  size_t lds = 0;
  // launch variant of the tile kernels: 0 per-slab only, 1 fixed only, 2 mixed
  int variant() const { return fixed ? 1 : anyfix ? 2 : 0; }
  void add(J j, long nb, bool fix = false) {
    fixed = fixed && fix;
    anyfix = anyfix || fix;
    j.block0 = blocks;
    blocks += nb;
    jobs.push_back(j);
  }
};

struct VCycle {
  std::vector<Site<TileJob>> down, up;   // by level l = 0 .. Lmax-2
  std::vector<Site<TileJob>> downp, upp;   // sweeps of the jobs with register-pencil fields, by level
  std::vector<Site<FuseJob>> fused;      // by fused top level index 0 .. Lmax-1
  Site<PointJob> tri;                    // exact 1-D solves
};

// VC_AX, VC_HX: the A and H cycles with their output stored to Xnu; VC_HA: the
// H cycle adding its result into its output (the last of nu > 1 H cycles)
enum { VC_A = 0, VC_H1 = 1, VC_H2 = 2, VC_AX = 3, VC_HX = 4, VC_HA = 5 };

struct Sites {
  Site<ResidJob> resid[2];
  VCycle vc[6];
  Site<TileJob> nu[2];   // steps between the cycles of an application with nu > 1 (A, H): b -= L x, o += x
  Site<TileJob> nures;   // b -= L o after the first of nu_H > 1 H cycles (tiled operator)
  Site<TileJob> mid;
  std::vector<Site<TimeJob>> a4, a6;
  std::vector<FinJob> fin;
  FinJob* fin_dev = nullptr;
};

// Optional per-launch device timing (HIP events on the context's stream).
// Phases of an iteration for the per-phase device times of a solve:
// residuals and stop test (a1, a3), A-tilde solves (a2), time transforms
// (a4, a6), H-blocks (a5), and everything else (GMRES orthogonalisation,
// casts, setup).
enum { PH_RESID = 0, PH_ATILDE = 1, PH_DST = 2, PH_HBLOCK = 3, PH_OTHER = 4, PH_COUNT = 5 };

struct KTimer {
  bool on = false;
  int level = 0;
  int phase = PH_OTHER;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    const char* name;
    int level;
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  const char* pend_name = nullptr;
  int pend_level = 0;
  int pend_phase = PH_OTHER;
  hipEvent_t pend_a = nullptr;
  struct Agg {
    std::string name;
    int level;
    long count;
    double ms;
  };
  std::vector<Agg> agg;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

struct SolverBase;

}  // namespace stpx

using namespace stpx;

struct stp_ctx {
  int P = 0, dim = 0, prec = 0, spatial = STP_SPATIAL_MG, rm = 1;
  int disc = STP_DISC_FD;
  stp_options opt{};
  hipStream_t stream = nullptr;
  std::vector<Problem> pr;
  void* ws = nullptr;
  bool own_ws = false;
  size_t tables_off = 0;
  size_t tables_bytes = 0;
  // setup and tuning scratch (omega estimate, kappa check, autotuner): a region
  // at the end of a caller's workspace, or (library-owned workspace) allocated
  // for the duration of each use
  double* scratch = nullptr;
  size_t scratch_n = 0;       // doubles the region holds (0: allocate per use)
  double t_setup_ms = 0, t_omega_ms = 0;
  DevState* state_host = nullptr;   // pinned, P entries
  Sites sites;
  SolverBase* impl = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  KTimer kt;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  // batch contexts: problems the launch tables cover (empty: all).  A solve
  // drops stopped problems from the tables at its host checks (their blocks
  // would only be dispatched to exit) and restores the full set at its end.
  std::vector<char> active;
  hipGraphExec_t gexecA = nullptr, gexecH = nullptr;   // A~^{-1} cycle and H~^{-1} (GMRES preconditioner)
  Schedule sched;
  std::string sched_text;
};

namespace stpx {
constexpr int kMaxNu = 8;   // V-cycles per spatial preconditioner application
// nu_A or nu_H > 1 with multigrid: the cycles of one application run through Xnu
inline bool multi_cycle(const stp_ctx* c) {
  return c->spatial == STP_SPATIAL_MG && (c->opt.nu_A > 1 || c->opt.nu_H > 1);
}
}  // namespace stpx

inline void kt_begin(stp_ctx* c, const char* name) {
  if (!c->kt.on) return;
  hipEvent_t a = c->kt.get();
  if (!a) return;
  (void)hipEventRecord(a, c->stream);
  c->kt.pend_name = name;
  c->kt.pend_level = c->kt.level;
  c->kt.pend_phase = c->kt.phase;
  c->kt.pend_a = a;
}

inline void kt_end(stp_ctx* c) {
  if (!c->kt.on || !c->kt.pend_name) return;
  hipEvent_t b = c->kt.get();
  if (b) {
    (void)hipEventRecord(b, c->stream);
    c->kt.recs.push_back({c->kt.pend_name, c->kt.pend_level, c->kt.pend_phase, c->kt.pend_a, b});
  }
  c->kt.pend_name = nullptr;
}

// Every kernel launch goes through KLAUNCH (optional timing) and LAUNCH_CHECK.
#define KLAUNCH_NAMED(name, kern, ...)     \
  do {                                     \
    kt_begin(&*c, name);                   \
    hipLaunchKernelGGL(kern, __VA_ARGS__); \
  } while (0)
#define KLAUNCH(kern, ...) KLAUNCH_NAMED(#kern, kern, __VA_ARGS__)

namespace stpx {

// ---------------------------------------------------------------------------
// typed execution
// ---------------------------------------------------------------------------
struct SolverBase {
  virtual ~SolverBase() {}
  virtual stp_status init() = 0;
  virtual stp_status launch_knob(int knob) = 0;
  virtual stp_status launch_transform(int g) = 0;
  virtual stp_status setup_problem(Problem& q) = 0;
  // full = false: only up to the stop test (the u-update of an iteration whose
  // stop test must fire would find the problem done and do nothing)
  virtual stp_status iteration(bool full = true) = 0;
  virtual stp_status run_vcycle(int which) = 0;
  virtual stp_status run_precH() = 0;
  virtual stp_status cast_in(const double* a, void* b, long n) = 0;
  // W1 of problem 0 = sgn (r + K^T d) in the storage type (input of the H-tilde solve)
  virtual stp_status kt_add_in(const double* r, const double* d, double sgn) = 0;
  virtual stp_status cast_out(const void* a, double scale, double* b, long n) = 0;
  virtual stp_status resid(int which) = 0;
};

// the typed solvers (stp_f64.hip, stp_f32.hip, stp_bf16.hip)
SolverBase* make_solver_f64(stp_ctx* c);
SolverBase* make_solver_f32(stp_ctx* c);
SolverBase* make_solver_bf16(stp_ctx* c);
// k_finalize (one block per problem) on the context stream
stp_status launch_finalize(stp_ctx* c);

}  // namespace stpx

// Host side of the space-time Uzawa solver: problem setup, multigrid
// hierarchy, workspace planning, the iteration driver and the C ABI of stp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "stp.h"
#include "stp_kernels.h"
#include "stp_tiles.h"

using namespace stp;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
struct stp_ctx;
static inline void kt_end(stp_ctx* c);

static stp_status fail(stp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

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

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace {

struct Level {
  int n;
  double h;
  Geom g;
  double* kraw;      // unscaled nodal fields (float64), R x nnodes
  void* kscaled;     // TC fields scaled by 0.5/h^2
  void *b, *x, *t, *e;  // TS work vectors (levels >= 1); x, t also on level 0
};

struct Bump {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  bool dry = true;
  void* take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    void* p = dry ? nullptr : base + off;
    off += bytes;
    return p;
  }
};

size_t ts_bytes(int prec) { return prec == STP_PREC_F64 ? 8 : (prec == STP_PREC_F32 ? 4 : 2); }
size_t tc_bytes(int prec) { return prec == STP_PREC_F64 ? 8 : 4; }

long ipow(long a, int d) {
  long r = 1;
  for (int i = 0; i < d; ++i) r *= a;
  return r;
}

dim3 grid_pts(long npts, int S) {
  const long bx = (npts + kBlock - 1) / kBlock;
  const int gy = std::min(S, 65535);
  const int gz = (S + 65534) / 65535;
  return dim3(unsigned(bx), unsigned(gy), unsigned(gz));
}

struct SolverBase;

// Optional per-launch device timing (HIP events on the context's stream).
struct KTimer {
  bool on = false;
  int level = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    const char* name;
    int level;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  const char* pend_name = nullptr;
  int pend_level = 0;
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

// Columns per block and LDS bytes of the FFT time transform (C = 0: use the dense path).
void fft_layout(int N, size_t tcb, int& C, size_t& lds) {
  C = 0;
  lds = 0;
  if (N < 1 || (N & (N - 1)) != 0 || N > 4096) return;
  C = std::max(1, std::min(16, 4096 / N));
  lds = (size_t(2) * N * C + size_t(4) * N) * tcb;
  if (lds > 160 * 1024) {
    C = 0;
    lds = 0;
  }
}

}  // namespace

struct stp_ctx {
  int dim = 0, n = 0, N = 0, R = 0;
  double tau = 0;
  stp_options opt{};
  int spatial = STP_SPATIAL_MG;
  double omega = 0.8;
  hipStream_t stream = nullptr;
  const double* F = nullptr;
  const double* u0 = nullptr;
  const double* fields = nullptr;
  std::vector<double> tcoef;   // R x N
  std::vector<double> abar;    // R
  std::vector<Level> lv;
  Geom g0{};
  // device memory
  void* ws = nullptr;
  bool own_ws = false;
  DevState* state = nullptr;
  DevState* state_host = nullptr;  // pinned
  double* partial = nullptr;
  long npartial = 0;               // capacity of the partial-sum buffer
  long npart_resid = 0;            // partials written by the residual kernel (tile grid)
  long npart_points = 0;           // partials written by point-grid reductions
  int sb_resid = 1;                // slabs per block of the residual kernels
  double* kap64 = nullptr;         // fine scaled fields, float64
  double* cA64 = nullptr;          // N x kMaxRank, tau*tcoef
  void* cA = nullptr;              // TC, N x kMaxRank
  void* sigH = nullptr;            // TC, N
  void* cH = nullptr;              // TC, N x kMaxRank
  void* cMid = nullptr;            // TC, kMaxRank
  void* sinT = nullptr;            // TC, N x N: sinT[k][n] = sin((2k+1)(n+1)pi/2N)  (Phi^{-T})
  void* sinM = nullptr;            // TC, N x N: sinM[n][k] = same value            (Phi^{-1})
  void* tw = nullptr;              // TC, 2N: exp(-2 pi i m / N)   (re block, im block)
  void* tw4 = nullptr;             // TC, 2N: exp(-i pi m / (2N))
  int fft_cols = 0;                // columns per block of the FFT path (0: dense path)
  size_t fft_lds = 0;
  void *W1 = nullptr, *W2 = nullptr;
  void* tri = nullptr;             // TC scratch for exact 1-D solves, 2 x N x n
  double fnorm = 0;
  SolverBase* impl = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  KTimer kt;
  // one Uzawa iteration captured as a HIP graph (valid for the (u, p) it was captured with)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* g_u = nullptr;
  double* g_p = nullptr;
};

static inline void kt_begin(stp_ctx* c, const char* name) {
  if (!c->kt.on) return;
  hipEvent_t a = c->kt.get();
  if (!a) return;
  (void)hipEventRecord(a, c->stream);
  c->kt.pend_name = name;
  c->kt.pend_level = c->kt.level;
  c->kt.pend_a = a;
}

static inline void kt_end(stp_ctx* c) {
  if (!c->kt.on || !c->kt.pend_name) return;
  hipEvent_t b = c->kt.get();
  if (b) {
    (void)hipEventRecord(b, c->stream);
    c->kt.recs.push_back({c->kt.pend_name, c->kt.pend_level, c->kt.pend_a, b});
  }
  c->kt.pend_name = nullptr;
}

// Every kernel launch goes through KLAUNCH (optional timing) and LAUNCH_CHECK.
#define KLAUNCH(kern, ...)                 \
  do {                                     \
    kt_begin(&*c, #kern);                  \
    hipLaunchKernelGGL(kern, __VA_ARGS__); \
  } while (0)
#define KLAUNCH_NAMED(name, kern, ...)     \
  do {                                     \
    kt_begin(&*c, name);                   \
    hipLaunchKernelGGL(kern, __VA_ARGS__); \
  } while (0)

namespace {

struct SolverBase {
  virtual ~SolverBase() {}
  virtual stp_status precA(const void* b, double* acc64, void* out) = 0;
  virtual stp_status precH(void* W1, void* W2, double* acc64, void* out, double alpha) = 0;
  virtual stp_status iteration(double* u, double* p) = 0;
  virtual stp_status setup_tables() = 0;
  virtual stp_status cast_in(const double* a, void* b, long n) = 0;
  virtual stp_status cast_out(const void* a, double* b, long n) = 0;
};

template <typename TS, typename TC>
struct Solver : SolverBase {
  stp_ctx* c;
  explicit Solver(stp_ctx* ctx) : c(ctx) {}

  TC omegaJ() const { return c->dim == 1 ? TC(2.0 / 3.0) : (c->dim == 2 ? TC(4.0 / 5.0) : TC(6.0 / 7.0)); }

  LevelOp fam(int l, int which) const {
    LevelOp L;
    L.kap = c->lv[l].kscaled;
    L.R = c->R;
    L.S = c->N;
    L.uniform = 0;
    if (which == 0) {          // A family: tau_n A_n
      L.sig = nullptr;
      L.c = c->cA;
    } else if (which == 1) {   // H family: mu_k I + tau A_ref
      L.sig = c->sigH;
      L.c = c->cH;
    } else {                   // middle: (2/N) tau A_ref
      L.sig = nullptr;
      L.c = c->cMid;
      L.uniform = 1;
    }
    return L;
  }

  const int* st() const { return &c->state->done; }

  // slabs per block for a launch over `tiles` tiles and S slabs: enough blocks
  // to fill the chip several times over, otherwise runs of up to 16 slabs
  static int pick_sb(long tiles, int S) {
    long sb = (tiles * S) / 2048;
    return int(std::max(1L, std::min(16L, sb)));
  }
  static dim3 grid_runs(long tiles, int S, int sb) {
    const long runs = (S + sb - 1) / sb;
    const long gy = std::min(runs, 65535L);
    const long gz = (runs + 65534) / 65535;
    return dim3(unsigned(tiles), unsigned(gy), unsigned(gz));
  }
  int rm() const { return c->R <= 1 ? 1 : (c->R <= 2 ? 2 : 4); }

  template <int D>
  stp_status vcycle_d(int l, int which, const TS* b, TS* out, double* acc64) {
    c->kt.level = l;
    Level& L = c->lv[l];
    const LevelOp op = fam(l, which);
    const int last = int(c->lv.size()) - 1;
    const int gy = std::min(c->N, 65535), gz = (c->N + 65534) / 65535;
    if (l == last) {
      // single-node level: x = b / D
      const long tot = long(c->N) * L.g.npts;
      const dim3 gr(unsigned((tot + kBlock - 1) / kBlock));
      if (acc64) {
        TS* tmp = (TS*)L.t;
        KLAUNCH((k_coarsest<D, TS, TC>), gr, dim3(kBlock), 0, c->stream, L.g, op, b, tmp, st());
        LAUNCH_CHECK();
        KLAUNCH((k_cast_add64<TS>), gr, dim3(kBlock), 0, c->stream, tot, (const TS*)tmp, acc64, st());
      } else {
        KLAUNCH((k_coarsest<D, TS, TC>), gr, dim3(kBlock), 0, c->stream, L.g, op, b, out, st());
      }
      LAUNCH_CHECK();
      return STP_OK;
    }
    Level& C = c->lv[l + 1];
    switch (rm()) {
      case 1: return vcycle_rm<D, 1>(l, which, op, L, C, b, out, acc64);
      case 2: return vcycle_rm<D, 2>(l, which, op, L, C, b, out, acc64);
      default: return vcycle_rm<D, 4>(l, which, op, L, C, b, out, acc64);
    }
  }

  template <int D, int RM>
  stp_status vcycle_rm(int l, int which, const LevelOp& op, Level& L, Level& C, const TS* b, TS* out, double* acc64) {
    const long td = tiles_for<D, DownTile<D>>(C.n);
    const int sbd = pick_sb(td, c->N);
    KLAUNCH((k_mg_down<D, TS, TC, RM>), grid_runs(td, c->N, sbd), dim3(kBlock), 0, c->stream, L.g, C.g, op, omegaJ(),
            b, (TS*)C.b, sbd, st());
    LAUNCH_CHECK();
    stp_status s = vcycle_d<D>(l + 1, which, (const TS*)C.b, (TS*)C.e, nullptr);
    if (s != STP_OK) return s;
    c->kt.level = l;
    const long tu = tiles_for<D, UpTile<D>>(L.n);
    const int sbu = pick_sb(tu, c->N);
    if (acc64)
      KLAUNCH((k_mg_up<D, TS, TC, RM, EPI_ADD64>), grid_runs(tu, c->N, sbu), dim3(kBlock), 0, c->stream, L.g, C.g, op,
              omegaJ(), b, (const TS*)C.e, (TS*)nullptr, acc64, sbu, st());
    else
      KLAUNCH((k_mg_up<D, TS, TC, RM, EPI_STORE>), grid_runs(tu, c->N, sbu), dim3(kBlock), 0, c->stream, L.g, C.g, op,
              omegaJ(), b, (const TS*)C.e, out, (double*)nullptr, sbu, st());
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status spatial_solve(int which, const TS* b, TS* out, double* acc64) {
    if (c->spatial == STP_SPATIAL_EXACT) {
      c->kt.level = 0;
      const LevelOp op = fam(0, which);
      const dim3 gr(unsigned((c->N + 63) / 64));
      if (acc64)
        KLAUNCH((k_tridiag<TS, TC, EPI_ADD64>), gr, dim3(64), 0, c->stream, c->lv[0].g, op, b, (TS*)nullptr,
                           acc64, (TC*)c->tri, st());
      else
        KLAUNCH((k_tridiag<TS, TC, EPI_STORE>), gr, dim3(64), 0, c->stream, c->lv[0].g, op, b, out,
                           (double*)nullptr, (TC*)c->tri, st());
      LAUNCH_CHECK();
      return STP_OK;
    }
    switch (c->dim) {
      case 1: return vcycle_d<1>(0, which, b, out, acc64);
      case 2: return vcycle_d<2>(0, which, b, out, acc64);
      default: return vcycle_d<3>(0, which, b, out, acc64);
    }
  }

  stp_status apply_mid(const TS* x, TS* y) {
    c->kt.level = 0;
    const LevelOp op = fam(0, 2);
    switch (c->dim) {
      case 1: return apply_mid_d<1>(op, x, y);
      case 2: return apply_mid_d<2>(op, x, y);
      default: return apply_mid_d<3>(op, x, y);
    }
  }

  template <int D>
  stp_status apply_mid_d(const LevelOp& op, const TS* x, TS* y) {
    const long tiles = tiles_for<D, UpTile<D>>(c->n);
    const int sb = pick_sb(tiles, c->N);
    const dim3 gr = grid_runs(tiles, c->N, sb);
    switch (rm()) {
      case 1: KLAUNCH((k_apply_tile<D, TS, TC, 1>), gr, dim3(kBlock), 0, c->stream, c->g0, op, x, y, sb, st()); break;
      case 2: KLAUNCH((k_apply_tile<D, TS, TC, 2>), gr, dim3(kBlock), 0, c->stream, c->g0, op, x, y, sb, st()); break;
      default: KLAUNCH((k_apply_tile<D, TS, TC, 4>), gr, dim3(kBlock), 0, c->stream, c->g0, op, x, y, sb, st()); break;
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  // out (or acc64 += alpha*) = T applied along time to in; mode 0: Phi^{-T}, 1: Phi^{-1}
  stp_status time_transform(int mode, const TS* in, TS* out, double* acc64, double alpha) {
    c->kt.level = 0;
    const long npts = c->g0.npts;
    if (c->N >= 4 && c->N <= 256 && (c->N & (c->N - 1)) == 0) {
      switch (c->N) {
        case 4: return fft2<1, 1>(mode, in, out, acc64, alpha);
        case 8: return fft2<2, 1>(mode, in, out, acc64, alpha);
        case 16: return fft2<2, 2>(mode, in, out, acc64, alpha);
        case 32: return fft2<3, 2>(mode, in, out, acc64, alpha);
        case 64: return fft2<3, 3>(mode, in, out, acc64, alpha);
        case 128: return fft2<4, 3>(mode, in, out, acc64, alpha);
        default: return fft2<4, 4>(mode, in, out, acc64, alpha);
      }
    }
    if (c->fft_cols > 0) {
      const int C = c->fft_cols;
      const dim3 gr(unsigned((npts + C - 1) / C));
      const size_t lds = c->fft_lds;
      const TC* tw = (const TC*)c->tw;
      const TC* tw4 = (const TC*)c->tw4;
      if (mode == 0)
        KLAUNCH((k_time_fft<TS, TC, MODE_A4, 0>), gr, dim3(kBlock), lds, c->stream, npts, c->N, C, tw, tw4,
                           in, out, (double*)nullptr, alpha, st());
      else if (acc64)
        KLAUNCH((k_time_fft<TS, TC, MODE_A6, 1>), gr, dim3(kBlock), lds, c->stream, npts, c->N, C, tw, tw4,
                           in, (TS*)nullptr, acc64, alpha, st());
      else
        KLAUNCH((k_time_fft<TS, TC, MODE_A6, 0>), gr, dim3(kBlock), lds, c->stream, npts, c->N, C, tw, tw4,
                           in, out, (double*)nullptr, alpha, st());
      LAUNCH_CHECK();
      return STP_OK;
    }
    const void* T = mode == 0 ? c->sinT : c->sinM;
    const int per_block = 4 * kDstKpt;
    const dim3 gr(unsigned((npts + 63) / 64), unsigned((c->N + per_block - 1) / per_block));
    if (acc64)
      KLAUNCH((k_time_dense<TS, TS, TC, 1>), gr, dim3(kBlock), 0, c->stream, npts, c->N, (const TC*)T, in,
                         (TS*)nullptr, acc64, alpha, st());
    else
      KLAUNCH((k_time_dense<TS, TS, TC, 0>), gr, dim3(kBlock), 0, c->stream, npts, c->N, (const TC*)T, in,
                         out, (double*)nullptr, alpha, st());
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int L1, int L2>
  stp_status fft2(int mode, const TS* in, TS* out, double* acc64, double alpha) {
    constexpr int C = kBlock / (1 << L1);
    const long npts = c->g0.npts;
    const dim3 gr(unsigned((npts + C - 1) / C));
    const size_t lds = size_t(1 << (L1 + L2)) * C * sizeof(TC);
    const TC* tw = (const TC*)c->tw;
    const TC* tw4 = (const TC*)c->tw4;
    if (mode == 0)
      KLAUNCH((k_time_fft2<TS, TC, MODE_A4, 0, L1, L2>), gr, dim3(kBlock), lds, c->stream, npts, tw, tw4, in, out,
              (double*)nullptr, alpha, st());
    else if (acc64)
      KLAUNCH((k_time_fft2<TS, TC, MODE_A6, 1, L1, L2>), gr, dim3(kBlock), lds, c->stream, npts, tw, tw4, in,
              (TS*)nullptr, acc64, alpha, st());
    else
      KLAUNCH((k_time_fft2<TS, TC, MODE_A6, 0, L1, L2>), gr, dim3(kBlock), lds, c->stream, npts, tw, tw4, in, out,
              (double*)nullptr, alpha, st());
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status precA(const void* b, double* acc64, void* out) override {
    return spatial_solve(0, (const TS*)b, (TS*)out, acc64);
  }

  // H-tilde^{-1}: W1 holds r (TS) on entry; result into acc64 (+= alpha * z) or out (TS).
  stp_status precH(void* W1v, void* W2v, double* acc64, void* out, double alpha) override {
    TS* W1 = (TS*)W1v;
    TS* W2 = (TS*)W2v;
    stp_status s;
    if ((s = time_transform(0, W1, W2, nullptr, 1.0)) != STP_OK) return s;          // rhat = Phi^{-T} r
    if ((s = spatial_solve(1, W2, W1, nullptr)) != STP_OK) return s;                  // x = H~_k^{-1} rhat
    if ((s = apply_mid(W1, W2)) != STP_OK) return s;                                  // y = (2/N) tau A x
    if ((s = spatial_solve(1, W2, W1, nullptr)) != STP_OK) return s;                  // yhat = H~_k^{-1} y
    return time_transform(1, W1, (TS*)out, acc64, alpha);                             // Phi^{-1} yhat
  }

  template <int D, int WHICH>
  stp_status resid_launch(const dim3& gr, const TimeOp& t, const double* u, const double* p, int sb) {
    double* part = WHICH == 1 ? c->partial : nullptr;
    const char* nm = WHICH == 0 ? "k_resid_tile<a1>" : "k_resid_tile<a3>";
    switch (rm()) {
      case 1: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, 1>), gr, dim3(kBlock), 0, c->stream, c->g0, t, c->tau, u, p, c->F, c->u0, (TS*)c->W1, part, sb, st()); break;
      case 2: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, 2>), gr, dim3(kBlock), 0, c->stream, c->g0, t, c->tau, u, p, c->F, c->u0, (TS*)c->W1, part, sb, st()); break;
      default: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, 4>), gr, dim3(kBlock), 0, c->stream, c->g0, t, c->tau, u, p, c->F, c->u0, (TS*)c->W1, part, sb, st()); break;
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int D>
  stp_status iteration_d(double* u, double* p) {
    c->kt.level = 0;
    const long tiles = tiles_for<D, UpTile<D>>(c->n);
    const int sb = c->sb_resid;
    const dim3 gr = grid_runs(tiles, c->N, sb);
    TimeOp t{c->kap64, c->cA64, c->R, c->N};
    stp_status s;
    if ((s = resid_launch<D, 0>(gr, t, u, p, sb)) != STP_OK) return s;
    s = spatial_solve(0, (const TS*)c->W1, nullptr, p);   // p += A~^{-1} r_p
    if (s != STP_OK) return s;
    c->kt.level = 0;
    if ((s = resid_launch<D, 1>(gr, t, u, p, sb)) != STP_OK) return s;
    KLAUNCH(k_finalize, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partial, c->npart_resid,
                       c->state, c->opt.tol, c->opt.max_iter);
    LAUNCH_CHECK();
    return precH(c->W1, c->W2, u, nullptr, c->omega);                  // u += omega H~^{-1} r_u
  }

  stp_status iteration(double* u, double* p) override {
    switch (c->dim) {
      case 1: return iteration_d<1>(u, p);
      case 2: return iteration_d<2>(u, p);
      default: return iteration_d<3>(u, p);
    }
  }

  stp_status cast_in(const double* a, void* b, long n) override {
    KLAUNCH((k_cast_from64<TS>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n,
                       a, (TS*)b);
    LAUNCH_CHECK();
    return STP_OK;
  }
  stp_status cast_out(const void* a, double* b, long n) override {
    KLAUNCH((k_cast_to64<TS>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n,
                       (const TS*)a, b);
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status setup_tables() override {
    const int N = c->N, R = c->R;
    if (c->fft_lds > 65536) {
      HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A4, 0>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(c->fft_lds)));
      HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A6, 0>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(c->fft_lds)));
      HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A6, 1>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(c->fft_lds)));
    }
    std::vector<TC> cA(size_t(N) * kMaxRank, TC(0)), cH(size_t(N) * kMaxRank, TC(0)), sig(N), mid(kMaxRank, TC(0));
    std::vector<double> cA64(size_t(N) * kMaxRank, 0.0);
    for (int s = 0; s < N; ++s)
      for (int r = 0; r < R; ++r) {
        cA64[size_t(s) * kMaxRank + r] = c->tau * c->tcoef[size_t(r) * N + s];
        cA[size_t(s) * kMaxRank + r] = TC(c->tau * c->tcoef[size_t(r) * N + s]);
        cH[size_t(s) * kMaxRank + r] = TC(c->tau * c->abar[r]);
      }
    for (int k = 0; k < N; ++k) sig[k] = TC(2.0 * std::sin((2.0 * k + 1.0) * M_PI / (4.0 * N)));
    for (int r = 0; r < R; ++r) mid[r] = TC((2.0 / N) * c->tau * c->abar[r]);
    std::vector<TC> sT(size_t(N) * N), sM(size_t(N) * N);
    for (int k = 0; k < N; ++k)
      for (int m = 0; m < N; ++m) {
        // sin((2k+1)(m+1) pi / (2N)) with the angle reduced exactly in integers
        const long q = (long(2 * k + 1) * long(m + 1)) % (4L * N);
        const double v = std::sin(double(q) * M_PI / (2.0 * N));
        sT[size_t(k) * N + m] = TC(v);   // row k (frequency), column m (time)
        sM[size_t(m) * N + k] = TC(v);   // row m (time), column k (frequency)
      }
    HIP_TRY(hipMemcpyAsync(c->cA64, cA64.data(), cA64.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->cA, cA.data(), cA.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->cH, cH.data(), cH.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->sigH, sig.data(), sig.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->cMid, mid.data(), mid.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    {
      double wd[32];
      float wf[32];
      for (int k = 0; k < 16; ++k) {
        wd[k] = std::cos(2.0 * M_PI * k / 16.0);
        wd[16 + k] = -std::sin(2.0 * M_PI * k / 16.0);
        wf[k] = float(wd[k]);
        wf[16 + k] = float(wd[16 + k]);
      }
      HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_w16d), wd, sizeof(wd)));
      HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_w16f), wf, sizeof(wf)));
    }
    if (c->fft_cols > 0) {
      std::vector<TC> tw(2 * size_t(N)), tw4(2 * size_t(N));
      for (int m = 0; m < N; ++m) {
        tw[m] = TC(std::cos(2.0 * M_PI * m / N));
        tw[N + m] = TC(-std::sin(2.0 * M_PI * m / N));
        tw4[m] = TC(std::cos(M_PI * m / (2.0 * N)));
        tw4[N + m] = TC(-std::sin(M_PI * m / (2.0 * N)));
      }
      HIP_TRY(hipMemcpyAsync(c->tw, tw.data(), tw.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(c->tw4, tw4.data(), tw4.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));   // host vectors go out of scope
    } else {
      HIP_TRY(hipMemcpyAsync(c->sinT, sT.data(), sT.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(c->sinM, sM.data(), sM.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    }
    // level fields: restrict unscaled float64 fields, then scale by 0.5/h^2 into TC
    for (size_t l = 0; l < c->lv.size(); ++l) {
      Level& L = c->lv[l];
      const long nn = L.g.nnodes;
      if (l > 0) {
        Level& F = c->lv[l - 1];
        for (int r = 0; r < R; ++r) {
          const dim3 gr(unsigned((nn + kBlock - 1) / kBlock));
          switch (c->dim) {
            case 1: KLAUNCH(k_restrict_kappa<1>, gr, dim3(kBlock), 0, c->stream, F.n, L.n, F.kraw + r * F.g.nnodes, L.kraw + r * nn); break;
            case 2: KLAUNCH(k_restrict_kappa<2>, gr, dim3(kBlock), 0, c->stream, F.n, L.n, F.kraw + r * F.g.nnodes, L.kraw + r * nn); break;
            default: KLAUNCH(k_restrict_kappa<3>, gr, dim3(kBlock), 0, c->stream, F.n, L.n, F.kraw + r * F.g.nnodes, L.kraw + r * nn); break;
          }
          LAUNCH_CHECK();
        }
      }
      const double sc = 0.5 / (L.h * L.h);
      const long tot = nn * R;
      KLAUNCH((k_scale_copy<TC>), dim3(unsigned((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
                         tot, (const double*)L.kraw, sc, (TC*)L.kscaled);
      LAUNCH_CHECK();
      if (l == 0) {
        KLAUNCH((k_scale_copy<double>), dim3(unsigned((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           c->stream, tot, (const double*)L.kraw, sc, c->kap64);
        LAUNCH_CHECK();
      }
    }
    return STP_OK;
  }
};

// Plan (dry run) or carve (real run) the workspace.
size_t plan(stp_ctx* c, Bump& bp) {
  const int prec = c->opt.precision;
  const size_t tsb = ts_bytes(prec), tcb = tc_bytes(prec);
  fft_layout(c->N, tcb, c->fft_cols, c->fft_lds);
  const long N = c->N;
  c->state = (DevState*)bp.take(sizeof(DevState));
  {
    long tiles = c->dim == 1 ? tiles_for<1, UpTile<1>>(c->n)
                 : c->dim == 2 ? tiles_for<2, UpTile<2>>(c->n) : tiles_for<3, UpTile<3>>(c->n);
    const dim3 gp = grid_pts(c->g0.npts, c->N);   // the setup reduction uses the point grid
    const long gyz = long(std::min(c->N, 65535)) * ((c->N + 65534) / 65535);
    {
      long sb = (tiles * c->N) / 2048;
      c->sb_resid = int(std::max(1L, std::min(16L, sb)));
    }
    const long runs = (c->N + c->sb_resid - 1) / c->sb_resid;
    c->npart_resid = tiles * std::min(runs, 65535L) * ((runs + 65534) / 65535);
    (void)gyz;
    c->npart_points = long(gp.x) * gp.y * gp.z;
    c->npartial = std::max(c->npart_resid, c->npart_points);
  }
  c->partial = (double*)bp.take(size_t(c->npartial) * 8);
  c->kap64 = (double*)bp.take(size_t(c->R) * c->g0.nnodes * 8);
  c->cA64 = (double*)bp.take(size_t(N) * kMaxRank * 8);
  c->cA = bp.take(size_t(N) * kMaxRank * tcb);
  c->cH = bp.take(size_t(N) * kMaxRank * tcb);
  c->sigH = bp.take(size_t(N) * tcb);
  c->cMid = bp.take(size_t(kMaxRank) * tcb);
  if (c->fft_cols > 0) {
    c->tw = bp.take(size_t(2) * N * tcb);
    c->tw4 = bp.take(size_t(2) * N * tcb);
  } else {
    c->sinT = bp.take(size_t(N) * N * tcb);
    c->sinM = bp.take(size_t(N) * N * tcb);
  }
  c->W1 = bp.take(size_t(N) * c->g0.npts * tsb);
  c->W2 = bp.take(size_t(N) * c->g0.npts * tsb);
  if (c->spatial == STP_SPATIAL_EXACT) c->tri = bp.take(size_t(2) * N * c->n * tcb);
  for (size_t l = 0; l < c->lv.size(); ++l) {
    Level& L = c->lv[l];
    L.kraw = (l == 0) ? nullptr : (double*)bp.take(size_t(c->R) * L.g.nnodes * 8);
    L.kscaled = bp.take(size_t(c->R) * L.g.nnodes * tcb);
    const size_t vb = size_t(N) * L.g.npts * tsb;
    if (c->spatial == STP_SPATIAL_EXACT || c->spatial == STP_SPATIAL_NONE) {
      L.b = L.x = L.t = L.e = nullptr;
      continue;
    }
    const bool last = (l + 1 == c->lv.size());
    L.b = (l == 0) ? nullptr : bp.take(vb);
    L.e = (l == 0) ? nullptr : bp.take(vb);
    L.x = nullptr;
    L.t = (last && l == 0) ? bp.take(vb) : nullptr;   // single-level hierarchy: scratch for the coarse solve
  }
  return bp.off + 256;
}

stp_status build_levels(stp_ctx* c) {
  c->lv.clear();
  int n = c->n;
  while (true) {
    Level L{};
    L.n = n;
    L.h = 1.0 / (n + 1);
    L.g.n = n;
    L.g.npts = ipow(n, c->dim);
    L.g.nnodes = ipow(n + 2, c->dim);
    c->lv.push_back(L);
    if (c->spatial == STP_SPATIAL_EXACT || c->spatial == STP_SPATIAL_NONE || n == 1) break;
    if (n % 2 == 0) return fail(STP_EUNSUPPORTED, "multigrid needs n = 2^L - 1 interior nodes per axis (got %d)", c->n);
    n = (n - 1) / 2;
    if (int(c->lv.size()) >= STP_MAX_LEVELS) return fail(STP_EUNSUPPORTED, "too many multigrid levels");
  }
  c->g0 = c->lv[0].g;
  return STP_OK;
}

stp_status validate(const stp_grid* g, int N, double tau, const stp_kappa* kappa, const double* F, const double* u0,
                    const stp_options* opt) {
  if (!g || !kappa || !opt) return fail(STP_EINVAL, "NULL grid, kappa or options");
  if (g->dim < 1 || g->dim > 3) return fail(STP_EINVAL, "dim must be 1, 2 or 3 (got %d)", g->dim);
  if (g->n < 1) return fail(STP_EINVAL, "n must be >= 1 (got %d)", g->n);
  if (N < 1) return fail(STP_EINVAL, "N must be >= 1 (got %d)", N);
  if (!(tau > 0) || !std::isfinite(tau)) return fail(STP_EINVAL, "tau must be finite and > 0");
  if (kappa->rank < 1 || kappa->rank > STP_MAX_RANK) return fail(STP_EINVAL, "kappa rank must be 1..%d", STP_MAX_RANK);
  if (!kappa->fields || !kappa->tcoef) return fail(STP_EINVAL, "NULL kappa fields or tcoef");
  if (!F || !u0) return fail(STP_EINVAL, "NULL F or u0");
  if (opt->precision < STP_PREC_F64 || opt->precision > STP_PREC_BF16) return fail(STP_EINVAL, "bad precision");
  if (opt->nu_A != 1 || opt->nu_H != 1) return fail(STP_EUNSUPPORTED, "only nu_A = nu_H = 1 is implemented");
  if (opt->spatial < STP_SPATIAL_AUTO || opt->spatial > STP_SPATIAL_NONE) return fail(STP_EINVAL, "bad spatial mode");
  if (opt->spatial == STP_SPATIAL_EXACT && g->dim != 1) return fail(STP_EUNSUPPORTED, "exact spatial solves are 1-D only");
  if (!(opt->tol >= 0)) return fail(STP_EINVAL, "tol must be >= 0");
  if (opt->max_iter < 0) return fail(STP_EINVAL, "max_iter must be >= 0");
  long npts = ipow(g->n, g->dim);
  if (double(npts) * double(N) > 4.0e12) return fail(STP_EINVAL, "problem too large");
  return STP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void stp_default_options(stp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = STP_PREC_F64;
  o->spatial = STP_SPATIAL_AUTO;
  o->nu_A = o->nu_H = 1;
  o->omega = 0.8;
  o->tol = 1e-8;
  o->max_iter = 500;
  o->kref_coef = nullptr;
  o->check_every = 8;
  o->use_graph = 1;
}

const char* stp_status_string(stp_status s) {
  switch (s) {
    case STP_OK: return "ok";
    case STP_EINVAL: return "invalid argument";
    case STP_ENOMEM: return "out of memory";
    case STP_EDEVICE: return "device error";
    case STP_ENOTCONV: return "not converged";
    case STP_EDIVERGED: return "diverged";
    case STP_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* stp_last_error(void) { return g_last_error.c_str(); }

static int resolve_spatial(int dim, int spatial) {
  if (spatial == STP_SPATIAL_AUTO) return dim == 1 ? STP_SPATIAL_EXACT : STP_SPATIAL_MG;
  return spatial;
}

size_t stp_workspace_bytes(const stp_grid* g, int N, int rank, const stp_options* opt) {
  if (!g || !opt || g->dim < 1 || g->dim > 3 || g->n < 1 || N < 1 || rank < 1 || rank > STP_MAX_RANK) return 0;
  stp_ctx c;
  c.dim = g->dim;
  c.n = g->n;
  c.N = N;
  c.R = rank;
  c.opt = *opt;
  c.spatial = resolve_spatial(g->dim, opt->spatial);
  if (build_levels(&c) != STP_OK) return 0;
  Bump bp;
  return plan(&c, bp);
}

stp_status stp_create(stp_ctx** out, const stp_grid* g, int N, double tau, const stp_kappa* kappa, const double* F,
                      const double* u0, const stp_options* opt_in, void* workspace, size_t ws_bytes,
                      void* hip_stream) {
  if (!out) return fail(STP_EINVAL, "NULL output context pointer");
  *out = nullptr;
  stp_options opt;
  if (opt_in) opt = *opt_in;
  else stp_default_options(&opt);
  stp_status s = validate(g, N, tau, kappa, F, u0, &opt);
  if (s != STP_OK) return s;
  std::unique_ptr<stp_ctx> c(new stp_ctx());
  c->dim = g->dim;
  c->n = g->n;
  c->N = N;
  c->R = kappa->rank;
  c->tau = tau;
  c->opt = opt;
  c->spatial = resolve_spatial(g->dim, opt.spatial);
  c->omega = opt.omega > 0 ? opt.omega : 0.8;
  c->stream = (hipStream_t)hip_stream;
  c->F = F;
  c->u0 = u0;
  c->fields = kappa->fields;
  c->tcoef.assign(kappa->tcoef, kappa->tcoef + size_t(c->R) * N);
  c->abar.assign(c->R, 0.0);
  if (opt.kref_coef) {
    for (int r = 0; r < c->R; ++r) c->abar[r] = opt.kref_coef[r];
  } else {
    for (int r = 0; r < c->R; ++r) {
      double sum = 0;
      for (int n = 0; n < N; ++n) sum += c->tcoef[size_t(r) * N + n];
      c->abar[r] = sum / N;
    }
  }
  if ((s = build_levels(c.get())) != STP_OK) return s;
  Bump dry;
  const size_t need = plan(c.get(), dry);
  if (workspace) {
    if (ws_bytes < need) return fail(STP_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(STP_EINVAL, "workspace not 256-byte aligned");
    c->ws = workspace;
  } else {
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(STP_ENOMEM, "hipMalloc of %zu bytes failed", need);
    }
    c->own_ws = true;
  }
  Bump real;
  real.dry = false;
  real.base = (char*)c->ws;
  real.cap = need;
  plan(c.get(), real);
  c->lv[0].kraw = const_cast<double*>(c->fields);  // level 0 reads the caller's fields
  HIP_TRY(hipHostMalloc((void**)&c->state_host, sizeof(DevState), hipHostMallocDefault));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  switch (opt.precision) {
    case STP_PREC_F64: c->impl = new Solver<double, double>(c.get()); break;
    case STP_PREC_F32: c->impl = new Solver<float, float>(c.get()); break;
    default: c->impl = new Solver<bf16, float>(c.get()); break;
  }
  if ((s = c->impl->setup_tables()) != STP_OK) return s;
  // kappa(t_n, x) > 0 at every node and step, and for the reference coefficient
  {
    const long nn = c->g0.nnodes;
    const long nb = (nn + kBlock - 1) / kBlock;
    std::vector<double> cref(kMaxRank, 0.0);
    for (int r = 0; r < c->R; ++r) cref[r] = c->abar[r];
    double* dref = (double*)c->partial;                    // reuse partials as scratch
    if (c->npartial < nb + kMaxRank) {
      // not enough scratch: use a temporary allocation
      HIP_TRY(hipMallocAsync((void**)&dref, size_t(nb + kMaxRank) * 8, c->stream));
    }
    double* part = dref + kMaxRank;
    HIP_TRY(hipMemcpyAsync(dref, cref.data(), kMaxRank * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<double> h(nb);
    double mn = 1e300;
    for (int pass = 0; pass < 2; ++pass) {
      const double* coef = pass == 0 ? c->cA64 : dref;
      KLAUNCH(k_kappa_min, dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, nn, c->R, pass == 0 ? N : 1,
                         c->fields, coef, part);
      LAUNCH_CHECK();
      HIP_TRY(hipMemcpyAsync(h.data(), part, size_t(nb) * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      mn = std::min(mn, *std::min_element(h.begin(), h.end()));
    }
    if (dref != c->partial) HIP_TRY(hipFreeAsync(dref, c->stream));
    if (!(mn > 0)) return fail(STP_EINVAL, "kappa must be > 0 at every node and step (min %.3e)", mn);
  }
  // ||f||
  {
    const dim3 gr = grid_pts(c->g0.npts, N);
    KLAUNCH(k_fnorm, gr, dim3(kBlock), 0, c->stream, c->g0, N, tau, F, u0, c->partial);
    LAUNCH_CHECK();
    KLAUNCH(k_sum_to, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partial, c->npart_points,
                       &c->state->fnorm);
    LAUNCH_CHECK();
    DevState hs{};
    HIP_TRY(hipMemcpyAsync(&hs, c->state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->fnorm = std::sqrt(hs.fnorm);
  }
  *out = c.release();
  return STP_OK;
}

void stp_destroy(stp_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  delete c->impl;
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->state_host) (void)hipHostFree(c->state_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->kt.pool) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

stp_status stp_apply_operator(stp_ctx* c, int op, const double* x, double* y) {
  if (!c || !x || !y) return fail(STP_EINVAL, "NULL argument");
  const dim3 gr = grid_pts(c->g0.npts, c->N);
  TimeOp t{c->kap64, c->cA64, c->R, c->N};
  const long nv = long(c->N) * c->g0.npts;
  if (op == STP_OP_B) {
    switch (c->dim) {
      case 1: KLAUNCH(k_apply_B<1>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, y); break;
      case 2: KLAUNCH(k_apply_B<2>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, y); break;
      default: KLAUNCH(k_apply_B<3>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, y); break;
    }
  } else if (op == STP_OP_SADDLE) {
    switch (c->dim) {
      case 1: KLAUNCH(k_apply_saddle<1>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, x + nv, y, y + nv); break;
      case 2: KLAUNCH(k_apply_saddle<2>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, x + nv, y, y + nv); break;
      default: KLAUNCH(k_apply_saddle<3>, gr, dim3(kBlock), 0, c->stream, c->g0, t, x, x + nv, y, y + nv); break;
    }
  } else {
    return fail(STP_EINVAL, "unknown operator %d", op);
  }
  LAUNCH_CHECK();
  return STP_OK;
}

stp_status stp_apply_precond(stp_ctx* c, int which, const double* r, double* z) {
  if (!c || !r || !z) return fail(STP_EINVAL, "NULL argument");
  if (which != STP_PC_A && which != STP_PC_H) return fail(STP_EINVAL, "unknown preconditioner %d", which);
  if (c->spatial == STP_SPATIAL_NONE) return fail(STP_EUNSUPPORTED, "context created without a spatial solver");
  const long nv = long(c->N) * c->g0.npts;
  // the state flag must read "running" for the kernels to execute
  HIP_TRY(hipMemsetAsync(c->state, 0, sizeof(int) * 2, c->stream));
  stp_status s;
  if ((s = c->impl->cast_in(r, c->W1, nv)) != STP_OK) return s;
  if (which == STP_PC_A) {
    HIP_TRY(hipMemsetAsync(z, 0, size_t(nv) * 8, c->stream));
    return c->impl->precA(c->W1, z, nullptr);
  }
  HIP_TRY(hipMemsetAsync(z, 0, size_t(nv) * 8, c->stream));
  return c->impl->precH(c->W1, c->W2, z, nullptr, 1.0);
}

// Capture one iteration on a private stream (capture is not possible on the
// null stream); the instantiated graph is replayed on the context's stream.
static stp_status capture_iteration(stp_ctx* c, double* u, double* p) {
  if (c->gexec && c->g_u == u && c->g_p == p) return STP_OK;
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  c->stream = c->cap_stream;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  stp_status s = STP_OK;
  if (e == hipSuccess) {
    s = c->impl->iteration(u, p);
    e = hipStreamEndCapture(c->cap_stream, &graph);
  }
  c->stream = saved;
  if (s != STP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(STP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return fail(STP_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  c->g_u = u;
  c->g_p = p;
  return STP_OK;
}

stp_status stp_uzawa_solve(stp_ctx* c, double* u, double* p, stp_stats* stats) {
  if (!c || !u || !p) return fail(STP_EINVAL, "NULL argument (u and p are required)");
  if (c->spatial == STP_SPATIAL_NONE) return fail(STP_EUNSUPPORTED, "context created without a spatial solver");
  DevState init{};
  init.fnorm = c->fnorm;
  HIP_TRY(hipMemcpyAsync(c->state, &init, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  const int chunk = std::max(1, c->opt.check_every);
  stp_status s = STP_OK;
  int launched = 0;
  DevState hs{};
  const int max_launch = c->opt.max_iter + 1;   // iterations 0..max_iter each evaluate the stop test
  const bool graph = c->opt.use_graph && !c->kt.on;
  if (graph && (s = capture_iteration(c, u, p)) != STP_OK) return s;
  while (true) {
    const int todo = std::min(chunk, max_launch - launched);
    for (int q = 0; q < todo; ++q) {
      if (graph) HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
      else if ((s = c->impl->iteration(u, p)) != STP_OK) return s;
      ++launched;
    }
    HIP_TRY(hipMemcpyAsync(c->state_host, c->state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    hs = *c->state_host;
    if (hs.done) break;
    if (launched >= max_launch) return fail(STP_EDEVICE, "iteration state did not terminate");
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  HIP_TRY(hipEventSynchronize(c->ev1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  stp_status res = hs.done == 1 ? STP_OK : (hs.done == 2 ? STP_EDIVERGED : STP_ENOTCONV);
  if (stats) {
    stats->iters = hs.iter;
    stats->rel_res = hs.rel;
    stats->omega_used = c->omega;
    stats->t_solve_ms = ms;
    stats->status = res;
  }
  if (res == STP_EDIVERGED) fail(res, "residual diverged at iteration %d (rel %.3e)", hs.iter, hs.rel);
  if (res == STP_ENOTCONV) fail(res, "max_iter %d reached (rel %.3e)", c->opt.max_iter, hs.rel);
  return res;
}

stp_status stp_timing_enable(stp_ctx* c, int enable) {
  if (!c) return fail(STP_EINVAL, "NULL context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->kt.recs.clear();
  c->kt.agg.clear();
  c->kt.used = 0;
  c->kt.pend_name = nullptr;
  c->kt.on = enable != 0;
  return STP_OK;
}

int stp_timing_count(stp_ctx* c) {
  if (!c) return -1;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
  for (const auto& r : c->kt.recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    bool found = false;
    for (auto& a : c->kt.agg)
      if (a.level == r.level && a.name == r.name) {
        a.count += 1;
        a.ms += ms;
        found = true;
        break;
      }
    if (!found) c->kt.agg.push_back({std::string(r.name), r.level, 1, double(ms)});
  }
  c->kt.recs.clear();
  c->kt.used = 0;
  return int(c->kt.agg.size());
}

stp_status stp_timing_get(stp_ctx* c, int idx, const char** name, int* level, long* launches, double* total_ms) {
  if (!c || idx < 0 || idx >= int(c->kt.agg.size())) return fail(STP_EINVAL, "bad timing index");
  const auto& a = c->kt.agg[idx];
  if (name) *name = a.name.c_str();
  if (level) *level = a.level;
  if (launches) *launches = a.count;
  if (total_ms) *total_ms = a.ms;
  return STP_OK;
}

}  // extern "C"

// Device kernels of the space-time Uzawa solver (gfx950, wave64).
//
// Vectors are slab-major [s][z][y][x] on the n^d interior nodes; coefficient
// fields are nodal on the (n+2)^d nodes including the boundary.  Every kernel
// covers all time slabs in one launch: blockIdx.x walks the points of a slab,
// blockIdx.y (+ gridDim.y * blockIdx.z) the slabs.
//
// Operator of a slab s on a multigrid level:
//     L_s x = sigma_s x + sum_r c_{s,r} A(kappa_r) x,
// evaluated face by face with face weight w = sum_r c_{s,r} (k_r[i] + k_r[nb]),
// where k_r = kappa_r * 0.5 / h^2 is stored pre-scaled per level.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace stp {

constexpr int kMaxRank = 4;
constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------
struct bf16 {
  uint16_t v;
};

__device__ __forceinline__ float bf16_to_f(bf16 a) { return __uint_as_float(uint32_t(a.v) << 16); }
__device__ __forceinline__ bf16 f_to_bf16(float f) {
  // round to nearest even; NaN stays NaN
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{uint16_t((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{uint16_t(u >> 16)};
}

template <typename TC, typename TS> __device__ __forceinline__ TC ld(const TS* p, long i) { return TC(p[i]); }
template <> __device__ __forceinline__ float ld<float, bf16>(const bf16* p, long i) { return bf16_to_f(p[i]); }
template <> __device__ __forceinline__ double ld<double, bf16>(const bf16* p, long i) { return double(bf16_to_f(p[i])); }

template <typename TS, typename TC> __device__ __forceinline__ void st(TS* p, long i, TC v) { p[i] = TS(v); }
template <> __device__ __forceinline__ void st<bf16, float>(bf16* p, long i, float v) { p[i] = f_to_bf16(v); }
template <> __device__ __forceinline__ void st<bf16, double>(bf16* p, long i, double v) { p[i] = f_to_bf16(float(v)); }

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
struct Geom {
  int n;        // interior nodes per axis
  long npts;    // n^d
  long nnodes;  // (n+2)^d
};

__device__ __forceinline__ int slab_index() { return blockIdx.y + gridDim.y * blockIdx.z; }

// point index inside a slab (< n^d < 2^31) -> coordinates, in 32-bit arithmetic
template <int D>
__device__ __forceinline__ void decode(long i, int n, int& x, int& y, int& z) {
  const unsigned q = unsigned(i), un = unsigned(n);
  if (D == 1) {
    x = int(q); y = 0; z = 0;
  } else if (D == 2) {
    const unsigned yy = q / un;
    y = int(yy); x = int(q - yy * un); z = 0;
  } else {
    const unsigned yz = q / un;
    const unsigned zz = yz / un;
    x = int(q - yz * un);
    z = int(zz);
    y = int(yz - zz * un);
  }
}

template <int D>
__device__ __forceinline__ long node_of(int x, int y, int z, int n) {
  const long nn = n + 2;
  if (D == 1) return x + 1;
  if (D == 2) return (long(y) + 1) * nn + x + 1;
  return ((long(z) + 1) * nn + y + 1) * nn + x + 1;
}

// Per-slab operator table entry, read once per block (uniform).
// Pointers read from a job table are generic (flat) pointers to the compiler,
// and flat memory instructions count against both the vector-memory and the
// LDS wait counters, so every LDS wait would also wait for in-flight HBM
// loads.  Re-deriving each pointer from its integer value in the global
// address space makes the compiler emit global loads and stores.
template <typename T>
__device__ __forceinline__ T* gmem(T* p) {
  using U = typename std::remove_cv<T>::type;
  return (T*)((__attribute__((address_space(1))) U*)(uintptr_t)p);
}

template <typename TC>
struct SlabOp {
  TC sigma;
  TC c[kMaxRank];
};

template <typename TC>
__device__ __forceinline__ SlabOp<TC> load_op(const TC* sig, const TC* c, int s, int R) {
  SlabOp<TC> op;
  op.sigma = sig ? sig[s] : TC(0);
#pragma unroll
  for (int r = 0; r < kMaxRank; ++r) op.c[r] = (r < R) ? c[s * kMaxRank + r] : TC(0);
  return op;
}

template <typename TC>
__device__ __forceinline__ TC kmix(const TC* kap, long nnodes, long node, const SlabOp<TC>& op, int R) {
  TC k = op.c[0] * kap[node];
#pragma unroll
  for (int r = 1; r < kMaxRank; ++r)
    if (r < R) k += op.c[r] * kap[r * nnodes + node];
  return k;
}

// Stencil pieces at interior point (x,y,z): returns diag D and sum_nb w*x_nb.
template <int D, typename TC, typename TV>
__device__ __forceinline__ void stencil(const TV* __restrict__ xs, long i, int x, int y, int z, const Geom& g,
                                        const TC* __restrict__ kap, const SlabOp<TC>& op, int R, TC& diag,
                                        TC& offsum) {
  const int n = g.n;
  const long nn = n + 2;
  const long node = node_of<D>(x, y, z, n);
  const TC kc = kmix(kap, g.nnodes, node, op, R);
  TC dsum = op.sigma, osum = 0;
  // x neighbours
  {
    TC w = kc + kmix(kap, g.nnodes, node - 1, op, R);
    dsum += w;
    if (x > 0) osum += w * ld<TC>(xs, i - 1);
    w = kc + kmix(kap, g.nnodes, node + 1, op, R);
    dsum += w;
    if (x < n - 1) osum += w * ld<TC>(xs, i + 1);
  }
  if (D >= 2) {
    TC w = kc + kmix(kap, g.nnodes, node - nn, op, R);
    dsum += w;
    if (y > 0) osum += w * ld<TC>(xs, i - n);
    w = kc + kmix(kap, g.nnodes, node + nn, op, R);
    dsum += w;
    if (y < n - 1) osum += w * ld<TC>(xs, i + n);
  }
  if (D >= 3) {
    const long plane = long(n) * n;
    const long nplane = nn * nn;
    TC w = kc + kmix(kap, g.nnodes, node - nplane, op, R);
    dsum += w;
    if (z > 0) osum += w * ld<TC>(xs, i - plane);
    w = kc + kmix(kap, g.nnodes, node + nplane, op, R);
    dsum += w;
    if (z < n - 1) osum += w * ld<TC>(xs, i + plane);
  }
  diag = dsum;
  offsum = osum;
}

// Both stencil sums of one point for two vectors with the same operator:
// diag, sum_nb w a_nb and sum_nb w b_nb (face weights computed once).
template <int D>
__device__ __forceinline__ void stencil2(const double* __restrict__ a, const double* __restrict__ b, long i, int x,
                                         int y, int z, const Geom& g, const double* __restrict__ kap,
                                         const SlabOp<double>& op, int R, double& diag, double& oa, double& ob) {
  const int n = g.n;
  const long nn = n + 2;
  const long node = node_of<D>(x, y, z, n);
  const double kc = kmix(kap, g.nnodes, node, op, R);
  double dsum = op.sigma, sa = 0.0, sb = 0.0;
  auto face = [&](long dnode, long di, bool inside) {
    const double w = kc + kmix(kap, g.nnodes, node + dnode, op, R);
    dsum += w;
    if (inside) {
      sa += w * a[i + di];
      sb += w * b[i + di];
    }
  };
  face(-1, -1, x > 0);
  face(1, 1, x < n - 1);
  if (D >= 2) {
    face(-nn, -n, y > 0);
    face(nn, n, y < n - 1);
  }
  if (D >= 3) {
    face(-nn * nn, -long(n) * n, z > 0);
    face(nn * nn, long(n) * n, z < n - 1);
  }
  diag = dsum;
  oa = sa;
  ob = sb;
}

// Diagonal only.
template <int D, typename TC>
__device__ __forceinline__ TC diag_at(int x, int y, int z, const Geom& g, const TC* __restrict__ kap,
                                      const SlabOp<TC>& op, int R) {
  const int n = g.n;
  const long nn = n + 2;
  const long node = node_of<D>(x, y, z, n);
  const TC kc = kmix(kap, g.nnodes, node, op, R);
  TC dsum = op.sigma + TC(2 * D) * kc;
  dsum += kmix(kap, g.nnodes, node - 1, op, R) + kmix(kap, g.nnodes, node + 1, op, R);
  if (D >= 2) dsum += kmix(kap, g.nnodes, node - nn, op, R) + kmix(kap, g.nnodes, node + nn, op, R);
  if (D >= 3) dsum += kmix(kap, g.nnodes, node - nn * nn, op, R) + kmix(kap, g.nnodes, node + nn * nn, op, R);
  return dsum;
}

__device__ __forceinline__ int done_flag(const int* st) { return *st; }

// Block-wide sum of a double (wave64 shuffles + LDS), result valid in thread 0.
template <int NTH = kBlock>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[NTH / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NTH / 64; ++w) s += red[w];
  }
  return s;
}

// ---------------------------------------------------------------------------
// time-global operators (float64)
// ---------------------------------------------------------------------------
struct TimeOp {
  const double* kap;   // fine-level scaled fields (float64)
  const double* cA;    // N x kMaxRank: tau * tcoef (operator tau_n A_n)
  int R;
  int N;
};

// y = B x = K x + A x
template <int D>
__global__ void __launch_bounds__(kBlock) k_apply_B(Geom g, TimeOp t, const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= t.N || i >= g.npts) return;
  int px, py, pz;
  decode<D>(i, g.n, px, py, pz);
  const SlabOp<double> op = load_op<double>(nullptr, t.cA, s, t.R);
  const double* xs = x + long(s) * g.npts;
  double dg, off;
  stencil<D, double>(xs, i, px, py, pz, g, t.kap, op, t.R, dg, off);
  const double xc = xs[i];
  const double xprev = s > 0 ? xs[i - g.npts] : 0.0;
  y[long(s) * g.npts + i] = (xc - xprev) + (dg * xc - off);
}

// saddle [p;u] -> [A p - K u ; -K^T p - (K + K^T + A) u]
template <int D>
__global__ void __launch_bounds__(kBlock) k_apply_saddle(Geom g, TimeOp t, const double* __restrict__ p,
                                                         const double* __restrict__ u, double* __restrict__ yp,
                                                         double* __restrict__ yu) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= t.N || i >= g.npts) return;
  int px, py, pz;
  decode<D>(i, g.n, px, py, pz);
  const SlabOp<double> op = load_op<double>(nullptr, t.cA, s, t.R);
  const long o = long(s) * g.npts;
  double dg, offp, offu;
  stencil2<D>(p + o, u + o, i, px, py, pz, g, t.kap, op, t.R, dg, offp, offu);
  const double pc = p[o + i];
  const double uc = u[o + i];
  const double Ap = dg * pc - offp;
  const double Au = dg * uc - offu;
  const double um = s > 0 ? u[o - g.npts + i] : 0.0;
  const double up = s + 1 < t.N ? u[o + g.npts + i] : 0.0;
  const double pp = s + 1 < t.N ? p[o + g.npts + i] : 0.0;
  yp[o + i] = Ap - (uc - um);
  yu[o + i] = -(pc - pp) - (2.0 * uc - um - up) - Au;
}

// ||f||^2 partials (setup)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_fnorm(Geom g, int N, const double* __restrict__ taus,
                                                  const double* __restrict__ F, const double* __restrict__ u0,
                                                  double* __restrict__ partial) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double v = 0.0;
  if (s < N && i < g.npts) {
    double f = taus[s] * F[long(s) * g.npts + i];
    if (s == 0) f += u0[i];
    v = f * f;
  }
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
}
#endif

// Solver state shared by the iteration kernels and the host.
struct DevState {
  int done;       // 0 running, 1 converged, 2 diverged, 3 max_iter
  int iter;       // current iteration index j
  double rel;     // ||f - B u_j|| / ||f||  (||f - B u_j|| when f = 0)
  double fnorm;
  double res0;
  double rp2, ru2;   // ||r_p||^2, ||r_u||^2 of the returned pair (after a solve)
};

// Deterministic reduction of one problem's residual partials and its stop
// decision; block b handles job b.
struct FinJob {
  const double* partial;
  long count;
  DevState* st;
  double tol;
  int max_iter;
};

__device__ __forceinline__ FinJob to_global(FinJob j) {
  j.partial = gmem(j.partial);
  j.st = gmem(j.st);
  return j;
}

#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_finalize(const FinJob* __restrict__ jobs) {
  const FinJob J = to_global(jobs[blockIdx.x]);
  DevState* st = J.st;
  if (st->done) return;
  // four independent partial sums per thread keep four loads in flight
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  long q = threadIdx.x;
  for (; q + 3 * kBlock < J.count; q += 4 * kBlock) {
    v0 += J.partial[q];
    v1 += J.partial[q + kBlock];
    v2 += J.partial[q + 2 * kBlock];
    v3 += J.partial[q + 3 * kBlock];
  }
  for (; q < J.count; q += kBlock) v0 += J.partial[q];
  const double s = block_sum((v0 + v1) + (v2 + v3));
  if (threadIdx.x == 0) {
    const double res = sqrt(s);
    const double rel = st->fnorm > 0 ? res / st->fnorm : res;   // f = 0: absolute residual
    st->rel = rel;
    if (st->iter == 0) st->res0 = res;
    if (!(rel == rel) || rel > 1e300 || (st->iter > 0 && res > 1e8 * st->res0 && res > 1e8 * st->fnorm * J.tol)) {
      st->done = 2;
    } else if (rel <= J.tol) {
      st->done = 1;
    } else if (st->iter >= J.max_iter) {
      st->done = 3;
    } else {
      st->iter = st->iter + 1;
    }
  }
}
#endif

#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void k_sum_to(const double* __restrict__ partial, long count, double* out) {
  double v = 0.0;
  for (long q = threadIdx.x; q < count; q += kBlock) v += partial[q];
  const double s = block_sum(v);
  if (threadIdx.x == 0) *out = s;
}
#endif

// ---------------------------------------------------------------------------
// spatial kernels on a multigrid level (storage TS, compute TC)
// ---------------------------------------------------------------------------
// How the slab coefficient sum_r c_{s,r} k_r varies over the slabs:
enum CMode {
  CM_SLAB = 0,      // a row of c per slab
  CM_UNIFORM = 1,   // one row (row 0) for every slab; sigma (if any) still per slab
  CM_SCALE = 2      // rank 1: the field k_0 times the per-slab scalar c_{s,0}
};

struct LevelOp {
  const void* kap;     // scaled fields, TC
  const void* sig;     // per-slab sigma (TC) or null
  const void* c;       // per-slab coefficients, S x kMaxRank (TC)
  int R;
  int S;               // number of slabs
  int cmode;           // CMode
};

template <typename TC>
__device__ __forceinline__ SlabOp<TC> level_op(const LevelOp& L, int s) {
  const TC* sig = (const TC*)L.sig;
  const TC* c = (const TC*)L.c;
  SlabOp<TC> op = load_op<TC>(nullptr, c, L.cmode == CM_UNIFORM ? 0 : s, L.R);
  op.sigma = sig ? sig[s] : TC(0);
  return op;
}

// A fixed-field launch (cmode != CM_SLAB) stages k_fix = sum_r f_r k_r once per
// block and scales it per slab by gamma_s:  f = row 0 and gamma = 1 (uniform),
// or f = (1, 0, ...) and gamma_s = c_{s,0} (rank 1).
template <typename TC>
__device__ __forceinline__ TC fixed_coef(const LevelOp& L, int r) {
  if (L.cmode == CM_SCALE) return r == 0 ? TC(1) : TC(0);
  return ((const TC*)L.c)[r];
}
template <typename TC>
__device__ __forceinline__ TC slab_scale(const LevelOp& L, int s) {
  return L.cmode == CM_SCALE ? ((const TC*)L.c)[s * kMaxRank] : TC(1);
}


// Epilogue of the last smoothing sweep: write out, or add it into a float64 vector.
enum Epi { EPI_STORE = 0, EPI_ADD64 = 1, EPI_ADDTS = 2 };   // EPI_ADDTS: add into the TS output (pencils)

// ---------------------------------------------------------------------------
// merged launches
//
// A launch serves one or several independent problems (a batch).  Each
// problem's share is a job: its first block index in the launch, its sizes,
// operator rows, buffers and stop flag.  A block finds its job by binary
// search over the first-block indices (uniform, scalar work), so problems of
// different sizes run in one launch.
// ---------------------------------------------------------------------------
struct TileJob {        // multigrid level kernels and the tile operator
  long block0;
  int tiles;            // spatial tiles per slab
  int sb;               // slabs per block
  Geom gf, gc;          // level (gc: next coarser level)
  LevelOp op;
  const void* b;        // input (TS)
  const void* e;        // coarse correction (TS)
  void* out;            // output (TS)
  double* acc64;        // float64 target of EPI_ADD64
  const int* state;     // the problem's stop flag
  int addout;           // top-level output: 0 store, 1 add into out (up-sweep), -1 subtract from out (operator)
  const void* pk;       // register-pencil down-sweep: fixed field and its face sums at the fine
  const void* pd;       // level's interior nodes (TC), or null
  void* acc_ts;         // operator between two cycles: the stored output o (TS), o += x, or null
};

struct PointJob {       // exact 1-D solves
  long block0;
  long total;           // slabs * points (coarsest) or slabs (1-D solve)
  Geom g;
  LevelOp op;
  const void* b;
  void* out;
  double* acc64;
  void* scratch;
  const int* state;
};


struct TimeJob {        // transforms along the time axis
  long block0;
  long npts;
  int N;
  int bx;               // column blocks (dense transform)
  const void* tw;       // FFT twiddles (2N; Bluestein: 2M)
  const void* tw4;      // quarter-wave twiddles (2N)
  int M;                // Bluestein FFT length (power of two >= 2N - 1)
  const void* chirp;    // Bluestein chirp w^{n^2/2} (2N)
  const void* bhat;     // Bluestein kernel spectrum / M (2M)
  const void* T;        // dense matrix (N x N)
  void* fs;             // four-step scratch: 2 x N x npts TC (re, im)
  const void* in;
  void* out;
  double* acc64;
  double alpha;
  const int* state;
};

__device__ __forceinline__ LevelOp to_global(LevelOp L) {
  L.kap = gmem(L.kap);
  L.sig = gmem(L.sig);
  L.c = gmem(L.c);
  return L;
}
__device__ __forceinline__ TileJob to_global(TileJob j) {
  j.op = to_global(j.op);
  j.b = gmem(j.b);
  j.e = gmem(j.e);
  j.out = gmem(j.out);
  j.acc64 = gmem(j.acc64);
  j.state = gmem(j.state);
  j.pk = gmem(j.pk);
  j.pd = gmem(j.pd);
  j.acc_ts = gmem(j.acc_ts);
  return j;
}
__device__ __forceinline__ PointJob to_global(PointJob j) {
  j.op = to_global(j.op);
  j.b = gmem(j.b);
  j.out = gmem(j.out);
  j.acc64 = gmem(j.acc64);
  j.scratch = gmem(j.scratch);
  j.state = gmem(j.state);
  return j;
}
__device__ __forceinline__ TimeJob to_global(TimeJob j) {
  j.tw = gmem(j.tw);
  j.tw4 = gmem(j.tw4);
  j.chirp = gmem(j.chirp);
  j.bhat = gmem(j.bhat);
  j.T = gmem(j.T);
  j.fs = gmem(j.fs);
  j.in = gmem(j.in);
  j.out = gmem(j.out);
  j.acc64 = gmem(j.acc64);
  j.state = gmem(j.state);
  return j;
}
// Logical block index of a merged launch.  The hardware hands workgroups to the
// eight XCDs round-robin, and each XCD has its own L2; remapping so that XCD x
// runs the contiguous range [x q, (x + 1) q) of logical blocks (q = grid / 8,
// the tail unchanged) keeps neighbouring tiles and column chunks, which share
// halo and straddled cache lines, on one L2.
__device__ __forceinline__ long block_id() {
  const long nb = gridDim.x, b = blockIdx.x;
  const long q = nb >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

template <typename J>
__device__ __forceinline__ int find_job(const J* __restrict__ jobs, int njobs) {
  int lo = 0, hi = njobs - 1;
  const long b = block_id();
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Exact 1-D solve per slab (Thomas algorithm), one thread per slab, 64 per block.
template <typename TS, typename TC, int EPI>
__global__ void __launch_bounds__(64) k_tridiag(const PointJob* __restrict__ jobs, int njobs) {
  const PointJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  const int s = int((block_id() - J.block0) * 64 + threadIdx.x);
  const LevelOp L = J.op;
  if (s >= L.S) return;
  const Geom g = J.g;
  const int n = g.n;
  const SlabOp<TC> op = level_op<TC>(L, s);
  const TC* kap = (const TC*)L.kap;
  TC* scratch = (TC*)J.scratch;
  TC* cp = scratch + long(s) * n;                     // modified super-diagonal
  TC* yp = scratch + long(L.S) * n + long(s) * n;     // modified right-hand side
  const TS* bs = (const TS*)J.b + long(s) * n;
  // row i (0-based interior), node i+1: diag = sigma + w_left + w_right, off-diagonals -w
  TC wl = kmix(kap, g.nnodes, 0, op, L.R) + kmix(kap, g.nnodes, 1, op, L.R);
  TC prev_d = 0, prev_y = 0;
  for (int i = 0; i < n; ++i) {
    const TC kc = kmix(kap, g.nnodes, i + 1, op, L.R);
    const TC wr = kc + kmix(kap, g.nnodes, i + 2, op, L.R);
    const TC dg = op.sigma + wl + wr;
    const TC a = -wl;
    const TC cup = -wr;
    TC denom = dg;
    TC rhs = ld<TC>(bs, i);
    if (i > 0) {
      denom = dg - a * prev_d;
      rhs = rhs - a * prev_y;
    }
    prev_d = (i < n - 1) ? cup / denom : TC(0);
    prev_y = rhs / denom;
    cp[i] = prev_d;
    yp[i] = prev_y;
    wl = wr;
  }
  TC xv = 0;
  for (int i = n - 1; i >= 0; --i) {
    xv = yp[i] - (i < n - 1 ? cp[i] * xv : TC(0));
    const long o = long(s) * n + i;
    if (EPI == EPI_STORE) st<TS, TC>((TS*)J.out, o, xv);
    else J.acc64[o] += double(xv);
  }
}

// ---------------------------------------------------------------------------
// dense transform along the time axis:  out[k][i] (=|+=) alpha * sum_m T[k][m] in[m][i]
// ---------------------------------------------------------------------------
constexpr int kDstKpt = 8;   // outputs per thread

template <typename TS, typename TC, int ACC64>
__global__ void __launch_bounds__(kBlock) k_time_dense(const TimeJob* __restrict__ jobs, int njobs) {
  const TimeJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  const long lb = block_id() - J.block0;
  const int bxi = int(lb % J.bx), byi = int(lb / J.bx);
  const long npts = J.npts;
  const int N = J.N;
  const TC* T = (const TC*)J.T;
  const TS* in = (const TS*)J.in;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long i = long(bxi) * 64 + lane;
  const int k0 = (byi * 4 + wv) * kDstKpt;
  if (k0 >= N) return;
  TC acc[kDstKpt];
#pragma unroll
  for (int q = 0; q < kDstKpt; ++q) acc[q] = 0;
  if (i < npts) {
    for (int m = 0; m < N; ++m) {
      const TC v = ld<TC>(in, long(m) * npts + i);
#pragma unroll
      for (int q = 0; q < kDstKpt; ++q)
        if (k0 + q < N) acc[q] += T[long(k0 + q) * N + m] * v;
    }
#pragma unroll
    for (int q = 0; q < kDstKpt; ++q) {
      if (k0 + q >= N) break;
      const long o = long(k0 + q) * npts + i;
      if (ACC64) J.acc64[o] += J.alpha * double(acc[q]);
      else st<TS, TC>((TS*)J.out, o, TC(J.alpha) * acc[q]);
    }
  }
}

// ---------------------------------------------------------------------------
// fast transforms along time for N = 2^m (length-N complex FFT in LDS)
//
//   MODE_A4:  out[k] = sum_n sin((2k+1)(n+1) pi / 2N) in[n]            (Phi^{-T})
//             s_m = in[N-1-m] * w4^m,  W = FFT(s),  Y_{2m} = Re W_m,
//             Y_{2m+1} = Re W_{N-1-m},  out[k] = (-1)^k Y_k
//   MODE_A6:  out[n] = sum_k sin((2k+1)(n+1) pi / 2N) in[k]            (Phi^{-1})
//             z_k = (-1)^k in[k];  v_m = z_{2m}, v_{N-1-m} = z_{2m+1};
//             X = Re(w4^m FFT(v)_m);  out[n] = X_{N-1-n}
// with w4 = exp(-i pi / 2N).  The FFT is a Stockham autosort with radix-4
// stages (and one radix-2 stage when log2 N is odd); each block holds C
// columns (consecutive spatial points) of all N time samples in LDS.
// ---------------------------------------------------------------------------
enum { MODE_A4 = 0, MODE_A6 = 1 };

// one copy per translation unit (internal linkage), set by the solver's init
static __constant__ double c_w16d[32];   // re[0..16), im[16..32)
static __constant__ float c_w16f[32];

template <typename TC> __device__ __forceinline__ TC w16re(int k);
template <typename TC> __device__ __forceinline__ TC w16im(int k);
template <> __device__ __forceinline__ double w16re<double>(int k) { return c_w16d[k]; }
template <> __device__ __forceinline__ double w16im<double>(int k) { return c_w16d[16 + k]; }
template <> __device__ __forceinline__ float w16re<float>(int k) { return c_w16f[k]; }
template <> __device__ __forceinline__ float w16im<float>(int k) { return c_w16f[16 + k]; }

template <int P>
__host__ __device__ constexpr int brev(int i) {
  int r = 0;
  for (int b = 1, rb = P >> 1; b < P; b <<= 1, rb >>= 1)
    if (i & b) r |= rb;
  return r;
}

// in-register radix-2 DIT DFT of size P <= 16 (forward, exp(-2 pi i/P)), natural order out
template <int P, typename TC>
__device__ __forceinline__ void dft_reg(TC (&xr)[P], TC (&xi)[P]) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int j = brev<P>(i);
    if (j > i) {
      TC t = xr[i]; xr[i] = xr[j]; xr[j] = t;
      t = xi[i]; xi[i] = xi[j]; xi[j] = t;
    }
  }
#pragma unroll
  for (int half = 1; half < P; half <<= 1) {
#pragma unroll
    for (int base = 0; base < P; base += 2 * half) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int a = base + j, b = a + half;
        TC tr, ti;
        if (j == 0) {
          tr = xr[b]; ti = xi[b];
        } else {
          const int tw = j * (16 / (2 * half));
          const TC wr = w16re<TC>(tw), wi = w16im<TC>(tw);
          tr = xr[b] * wr - xi[b] * wi;
          ti = xr[b] * wi + xi[b] * wr;
        }
        xr[b] = xr[a] - tr; xi[b] = xi[a] - ti;
        xr[a] = xr[a] + tr; xi[a] = xi[a] + ti;
      }
    }
  }
}



template <typename TC, int R, int MAXB>
__device__ __forceinline__ void fft_stage(TC* re, TC* im, const TC* twr, const TC* twi, int N, int Ns, int C,
                                          int col, int jg, int G) {
  const int nb = N / R;
  TC orr[MAXB * R], oii[MAXB * R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = jg + b * G;
    if (j < nb) {
      const int k = j & (Ns - 1);
      TC vr[R], vi[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const TC ar = re[(j + r * nb) * C + col], ai = im[(j + r * nb) * C + col];
        if (r == 0) {
          vr[r] = ar; vi[r] = ai;
        } else {
          const int ti = (k * r) * (N / (Ns * R));
          const TC wr = twr[ti], wi = twi[ti];
          vr[r] = ar * wr - ai * wi;
          vi[r] = ar * wi + ai * wr;
        }
      }
      if constexpr (R == 2) {
        orr[b * R + 0] = vr[0] + vr[1]; oii[b * R + 0] = vi[0] + vi[1];
        orr[b * R + 1] = vr[0] - vr[1]; oii[b * R + 1] = vi[0] - vi[1];
      } else if constexpr (R == 8) {
        dft_reg<R, TC>(vr, vi);   // R-point DFT in registers, natural order
#pragma unroll
        for (int q = 0; q < R; ++q) {
          orr[b * R + q] = vr[q];
          oii[b * R + q] = vi[q];
        }
      } else {
        // radix-4 DFT with e^{-2 pi i/4} = -i
        const TC s0r = vr[0] + vr[2], s0i = vi[0] + vi[2];
        const TC d0r = vr[0] - vr[2], d0i = vi[0] - vi[2];
        const TC s1r = vr[1] + vr[3], s1i = vi[1] + vi[3];
        const TC d1r = vr[1] - vr[3], d1i = vi[1] - vi[3];
        orr[b * R + 0] = s0r + s1r; oii[b * R + 0] = s0i + s1i;
        orr[b * R + 2] = s0r - s1r; oii[b * R + 2] = s0i - s1i;
        // q = 1: d0 - i d1 ; q = 3: d0 + i d1
        orr[b * R + 1] = d0r + d1i; oii[b * R + 1] = d0i - d1r;
        orr[b * R + 3] = d0r - d1i; oii[b * R + 3] = d0i + d1r;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = jg + b * G;
    if (j < nb) {
      const int k = j & (Ns - 1);
      const int idxD = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        re[(idxD + q * Ns) * C + col] = orr[b * R + q];
        im[(idxD + q * Ns) * C + col] = oii[b * R + q];
      }
    }
  }
  __syncthreads();
}

// A length-N (power of two, N C <= 4096) Stockham FFT of C columns in LDS, with
// the largest radix (8, 4 or 2) that divides what is left: fewer passes through
// LDS (four for N = 2048 instead of six with radix 4; radix 16 would need more
// registers than it saves).
template <typename TC>
__device__ __forceinline__ void fft_stages(TC* re, TC* im, const TC* twr, const TC* twi, int N, int C, int col,
                                           int jg, int G) {
  int Ns = 1;
  while (Ns < N) {
    const int rem = N / Ns;
    if (rem % 8 == 0) {
      fft_stage<TC, 8, 2>(re, im, twr, twi, N, Ns, C, col, jg, G);
      Ns *= 8;
    } else if (rem % 4 == 0) {
      fft_stage<TC, 4, 4>(re, im, twr, twi, N, Ns, C, col, jg, G);
      Ns *= 4;
    } else {
      fft_stage<TC, 2, 8>(re, im, twr, twi, N, Ns, C, col, jg, G);
      Ns *= 2;
    }
  }
}

// tw: 2N values (re[0..N), im[0..N)) of w_N^m; tw4: same for w_{4N}^m.
template <typename TS, typename TC, int MODE, int ACC64>
__device__ __forceinline__ void time_fft_body(const TimeJob& J, int C, const TC* __restrict__ tw,
                                              const TC* __restrict__ tw4, const TS* __restrict__ in,
                                              TS* __restrict__ out, double* __restrict__ out64) {
  const long npts = J.npts;
  const int N = J.N;
  const double alpha = J.alpha;
  const long lb = block_id() - J.block0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* re = reinterpret_cast<TC*>(smem_raw);
  TC* im = re + N * C;
  TC* twr = im + N * C;
  TC* twi = twr + N;
  TC* t4r = twi + N;
  TC* t4i = t4r + N;
  const int t = threadIdx.x;
  for (int q = t; q < N; q += kBlock) {
    twr[q] = tw[q]; twi[q] = tw[N + q];
    t4r[q] = tw4[q]; t4i[q] = tw4[N + q];
  }
  __syncthreads();
  const int col = t % C, jg = t / C, G = kBlock / C;
  const long i = lb * C + col;
  const bool valid = (jg < G) && (i < npts);
  for (int n = jg; n < N; n += G) {
    const TC v = valid ? ld<TC>(in, long(n) * npts + i) : TC(0);
    if (MODE == MODE_A4) {
      const int m = N - 1 - n;
      re[m * C + col] = v * t4r[m];
      im[m * C + col] = v * t4i[m];
    } else {
      const int pos = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
      re[pos * C + col] = (n & 1) ? -v : v;
      im[pos * C + col] = TC(0);
    }
  }
  __syncthreads();
  fft_stages<TC>(re, im, twr, twi, N, C, col, jg, G);
  if (!valid) return;
  for (int n = jg; n < N; n += G) {
    TC v;
    if (MODE == MODE_A4) {
      const int m = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
      v = (n & 1) ? -re[m * C + col] : re[m * C + col];
    } else {
      const int m = N - 1 - n;
      v = t4r[m] * re[m * C + col] - t4i[m] * im[m * C + col];
    }
    const long o = long(n) * npts + i;
    if (ACC64) out64[o] += alpha * double(v);
    else st<TS, TC>(out, o, TC(alpha) * v);
  }
}

template <typename TS, typename TC, int MODE, int ACC64>
__global__ void __launch_bounds__(kBlock) k_time_fft(const TimeJob* __restrict__ jobs, int njobs, int C) {
  const TimeJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  time_fft_body<TS, TC, MODE, ACC64>(J, C, (const TC*)J.tw, (const TC*)J.tw4, (const TS*)J.in, (TS*)J.out, J.acc64);
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// large powers of two (N > 4096): the same mappings with the length-N FFT split
// as N = N1 N2 (four-step; N1 = 2^ceil(log2(N)/2), both <= 1024).  With
// n = N2 n1 + n2 and k = k1 + N1 k2,
//   W_k = sum_n2 w_N2^{n2 k2} [ w_N^{n2 k1} sum_n1 w_N1^{n1 k1} s_{N2 n1 + n2} ].
// Pass 0: gather s for one n2 and C columns (pre-map), length-N1 FFT in LDS,
//         twiddle w_N^{n2 k1}, store to the scratch at row k1 N2 + n2.
// Pass 1: load row block k1, length-N2 FFT in LDS, post-map W_k to its output
//         (each FFT value feeds exactly one output).
// Blocks of a job: ceil(npts / C) column blocks times N1 rows (pass 0 skips
// rows >= N2 when N1 = 2 N2).
// ---------------------------------------------------------------------------
__host__ __device__ inline int four_n1(int N) {
  int m = 0;
  while ((1 << m) < N) ++m;
  return 1 << ((m + 1) / 2);
}

template <typename TS, typename TC, int MODE, int PASS, int ACC64>
__device__ __forceinline__ void time_fft4_body(const TimeJob& J, int C) {
  const long npts = J.npts;
  const int N = J.N, N1 = four_n1(N), N2 = N / N1;
  const int L = PASS == 0 ? N1 : N2;        // length of this pass's FFTs
  const int stride = PASS == 0 ? N2 : N1;   // w_L^j = w_N^{j stride}
  const long ncb = (npts + C - 1) / C;
  const long lb = block_id() - J.block0;
  const int row = int(lb / ncb);            // pass 0: n2; pass 1: k1
  if (PASS == 0 && row >= N2) return;
  const long cb = lb - long(row) * ncb;
  const TC* tw = (const TC*)J.tw;
  const TC* tw4 = (const TC*)J.tw4;
  TC* fre = (TC*)J.fs;
  TC* fim = fre + long(N) * npts;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* re = reinterpret_cast<TC*>(smem_raw);
  TC* im = re + L * C;
  TC* twr = im + L * C;
  TC* twi = twr + L;
  const int t = threadIdx.x;
  for (int q = t; q < L; q += kBlock) {
    twr[q] = tw[long(q) * stride];
    twi[q] = tw[N + long(q) * stride];
  }
  const int col = t % C, jg = t / C, G = kBlock / C;
  const long i = cb * C + col;
  const bool valid = (jg < G) && (i < npts);
  for (int a = jg; a < L; a += G) {
    TC vr = 0, vi = 0;
    if (PASS == 0) {
      const int m = a * N2 + row;
      if (MODE == MODE_A4) {   // s_m = in[N-1-m] w4^m
        const TC v = valid ? ld<TC>((const TS*)J.in, long(N - 1 - m) * npts + i) : TC(0);
        vr = v * tw4[m];
        vi = v * tw4[N + m];
      } else {                 // v_m = in[2m] (m < N/2), -in[2(N-1-m)+1] (m >= N/2)
        const int n = m < N / 2 ? 2 * m : 2 * (N - 1 - m) + 1;
        const TC v = valid ? ld<TC>((const TS*)J.in, long(n) * npts + i) : TC(0);
        vr = m < N / 2 ? v : -v;
      }
    } else if (valid) {
      const long o = (long(row) * N2 + a) * npts + i;
      vr = fre[o];
      vi = fim[o];
    }
    re[a * C + col] = vr;
    im[a * C + col] = vi;
  }
  __syncthreads();
  fft_stages<TC>(re, im, twr, twi, L, C, col, jg, G);
  if (!valid) return;
  for (int a = jg; a < L; a += G) {
    const TC xr = re[a * C + col], xi = im[a * C + col];
    if (PASS == 0) {   // a = k1: twiddle w_N^{n2 k1}, scratch row k1 N2 + n2
      const int e = int((long(row) * a) & (N - 1));
      const TC wr = tw[e], wi = tw[N + e];
      const long o = (long(a) * N2 + row) * npts + i;
      fre[o] = xr * wr - xi * wi;
      fim[o] = xr * wi + xi * wr;
    } else {           // a = k2: W_m, m = k1 + N1 k2
      const int m = row + N1 * a;
      int n;
      TC v;
      if (MODE == MODE_A4) {
        n = m < N / 2 ? 2 * m : 2 * (N - 1 - m) + 1;
        v = m < N / 2 ? xr : -xr;
      } else {
        n = N - 1 - m;
        v = tw4[m] * xr - tw4[N + m] * xi;
      }
      const long o = long(n) * npts + i;
      if (ACC64) J.acc64[o] += J.alpha * double(v);
      else st<TS, TC>((TS*)J.out, o, TC(J.alpha) * v);
    }
  }
}

template <typename TS, typename TC, int MODE, int PASS, int ACC64>
__global__ void __launch_bounds__(kBlock) k_time_fft4(const TimeJob* __restrict__ jobs, int njobs, int C) {
  const TimeJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  time_fft4_body<TS, TC, MODE, PASS, ACC64>(J, C);
}

// any N (Bluestein): the length-N DFT of the MODE_A4 / MODE_A6 mappings above
// (valid for every N, with the even/odd split of A6 at ceil(N/2)) as a chirp
// convolution,  X_k = c_k sum_n (x_n c_n) conj(c_{k-n}),  c_n = w_N^{n^2/2} =
// exp(-i pi (n^2 mod 2N) / N),  evaluated with two length-M Stockham FFTs in
// LDS (M = 2^m >= 2N - 1): A = FFT(x c, zero padded), R = FFT(conj(A Bhat)),
// X_k = c_k conj(R_k), where Bhat = FFT(b) / M and b holds conj(c) wrapped
// around (b_m = b_{M-m} = conj(c_m), |m| < N).  Tables: tw = w_M^m (2M),
// chirp (2N), bhat (2M), tw4 as above.
// ---------------------------------------------------------------------------
template <typename TS, typename TC, int MODE, int ACC64>
__device__ __forceinline__ void time_bluestein_body(const TimeJob& J, int C, const TC* __restrict__ twM,
                                                    const TC* __restrict__ tw4, const TC* __restrict__ chirp,
                                                    const TC* __restrict__ bhat, const TS* __restrict__ in,
                                                    TS* __restrict__ out, double* __restrict__ out64) {
  const long npts = J.npts;
  const int N = J.N, M = J.M;
  const double alpha = J.alpha;
  const long lb = block_id() - J.block0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* re = reinterpret_cast<TC*>(smem_raw);
  TC* im = re + M * C;
  TC* twr = im + M * C;
  TC* twi = twr + M;
  const int t = threadIdx.x;
  for (int q = t; q < M; q += kBlock) {
    twr[q] = twM[q];
    twi[q] = twM[M + q];
  }
  const int col = t % C, jg = t / C, G = kBlock / C;
  const long i = lb * C + col;
  const bool valid = (jg < G) && (i < npts);
  const int half = (N + 1) / 2;
  // a_n = s_n c_n for n < N, zero up to M
  for (int n = jg; n < M; n += G) {
    TC ar = TC(0), ai = TC(0);
    if (valid && n < N) {
      TC sr, si;
      if (MODE == MODE_A4) {
        const TC v = ld<TC>(in, long(N - 1 - n) * npts + i);
        sr = v * tw4[n];
        si = v * tw4[N + n];
      } else {
        const bool even = n < half;
        const int row = even ? 2 * n : 2 * (N - 1 - n) + 1;
        const TC v = ld<TC>(in, long(row) * npts + i);
        sr = even ? v : -v;
        si = TC(0);
      }
      const TC cr = chirp[n], ci = chirp[N + n];
      ar = sr * cr - si * ci;
      ai = sr * ci + si * cr;
    }
    re[n * C + col] = ar;
    im[n * C + col] = ai;
  }
  __syncthreads();
  auto fft = [&]() { fft_stages<TC>(re, im, twr, twi, M, C, col, jg, G); };
  fft();
  // conj(A_m Bhat_m): the second forward FFT then yields M conj(ifft(A Bhat))
  for (int m = jg; m < M; m += G) {
    if (jg < G) {
      const TC xr = re[m * C + col], xi = im[m * C + col];
      const TC br = bhat[m], bi = bhat[M + m];
      re[m * C + col] = xr * br - xi * bi;
      im[m * C + col] = -(xr * bi + xi * br);
    }
  }
  __syncthreads();
  fft();
  // X_k = c_k conj(R_k), k < N
  for (int k = jg; k < N; k += G) {
    if (jg < G) {
      const TC rr = re[k * C + col], ri = -im[k * C + col];
      const TC cr = chirp[k], ci = chirp[N + k];
      re[k * C + col] = rr * cr - ri * ci;
      im[k * C + col] = rr * ci + ri * cr;
    }
  }
  __syncthreads();
  if (!valid) return;
  for (int n = jg; n < N; n += G) {
    TC v;
    if (MODE == MODE_A4) {
      const int m = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
      v = (n & 1) ? -re[m * C + col] : re[m * C + col];
    } else {
      const int m = N - 1 - n;
      v = tw4[m] * re[m * C + col] - tw4[N + m] * im[m * C + col];
    }
    const long o = long(n) * npts + i;
    if (ACC64) out64[o] += alpha * double(v);
    else st<TS, TC>(out, o, TC(alpha) * v);
  }
}

template <typename TS, typename TC, int MODE, int ACC64>
__global__ void __launch_bounds__(kBlock) k_time_bluestein(const TimeJob* __restrict__ jobs, int njobs, int C) {
  const TimeJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  time_bluestein_body<TS, TC, MODE, ACC64>(J, C, (const TC*)J.tw, (const TC*)J.tw4, (const TC*)J.chirp,
                                           (const TC*)J.bhat, (const TS*)J.in, (TS*)J.out, J.acc64);
}

// ---------------------------------------------------------------------------
// two-step ("four-step") FFT variant for N = N1 * N2 <= 256 (N1 = 2^L1 >= N2 = 2^L2):
//   step 1: thread (col, n2) runs an N1-point DFT in registers over the samples
//           x[N2 n1 + n2] loaded straight from global memory, then twiddles by
//           w_N^{n2 k1};
//   step 2: one transpose through LDS;
//   step 3: thread (col, k1) runs an N2-point DFT in registers and writes
//           X[k1 + N1 k2] straight to global memory.
// The pre/post-processing of MODE_A4 / MODE_A6 (see above) is folded into the
// load and store addressing.  c_w16 holds w_16^k (set by the host).
// ---------------------------------------------------------------------------
// tw / tw4: 2N tables as in k_time_fft.  Dynamic LDS: N * C * sizeof(TC)
// (real and imaginary parts pass through it one after the other).
template <typename TS, typename TC, int MODE, int ACC64, int L1, int L2>
__device__ __forceinline__ void time_fft2_body(const TimeJob& J, const TC* __restrict__ tw,
                                               const TC* __restrict__ tw4, const TS* __restrict__ in,
                                               TS* __restrict__ out, double* __restrict__ out64) {
  const long npts = J.npts;
  const double alpha = J.alpha;
  const long lb = block_id() - J.block0;
  constexpr int N1 = 1 << L1, N2 = 1 << L2, N = N1 * N2;
  constexpr int C = kBlock / N1;             // columns per block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* lds = reinterpret_cast<TC*>(smem_raw);  // [k1][n2][col]
  const int t = threadIdx.x;
  const int col = t % C, j = t / C;          // j = n2 (step 1, if < N2) or k1 (step 3)
  const long i = lb * C + col;
  const bool valid = i < npts;
  TC xr[N1], xi[N1];
  const bool act1 = j < N2;
  if (act1) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int m = N2 * n1 + j;             // FFT input index
      int row;
      TC sgn = TC(1);
      if (MODE == MODE_A4) {
        row = N - 1 - m;
      } else {
        if (m < N / 2) row = 2 * m;
        else { row = 2 * (N - 1 - m) + 1; sgn = TC(-1); }
      }
      const TC v = valid ? sgn * ld<TC>(in, long(row) * npts + i) : TC(0);
      if (MODE == MODE_A4) {
        xr[n1] = v * tw4[m];
        xi[n1] = v * tw4[N + m];
      } else {
        xr[n1] = v;
        xi[n1] = TC(0);
      }
    }
    dft_reg<N1, TC>(xr, xi);
    // twiddle w_N^{n2 k1}
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      const int q = (j * k1) & (N - 1);
      const TC wr = tw[q], wi = tw[N + q];
      const TC a = xr[k1], b = xi[k1];
      xr[k1] = a * wr - b * wi;
      xi[k1] = a * wi + b * wr;
    }
  }
  // transpose through LDS: real parts, then imaginary parts
  TC yr[N2], yi[N2];
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (act1) {
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) lds[(k1 * N2 + j) * C + col] = part == 0 ? xr[k1] : xi[k1];
    }
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const TC v = lds[(j * N2 + n2) * C + col];
      if (part == 0) yr[n2] = v;
      else yi[n2] = v;
    }
    __syncthreads();
  }
  if (N2 > 1) dft_reg<N2, TC>(yr, yi);
  if (!valid) return;
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    const int k = j + N1 * k2;               // FFT output index
    int row;
    TC v;
    if (MODE == MODE_A4) {
      if (k < N / 2) { row = 2 * k; v = yr[k2]; }
      else { row = 2 * (N - 1 - k) + 1; v = -yr[k2]; }
    } else {
      row = N - 1 - k;
      v = tw4[k] * yr[k2] - tw4[N + k] * yi[k2];
    }
    const long o = long(row) * npts + i;
    if (ACC64) out64[o] += alpha * double(v);
    else st<TS, TC>(out, o, TC(alpha) * v);
  }
}

template <typename TS, typename TC, int MODE, int ACC64, int L1, int L2>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_time_fft2(const TimeJob* __restrict__ jobs, int njobs) {
  const TimeJob J = to_global(jobs[find_job(jobs, njobs)]);
  if (J.state && done_flag(J.state)) return;
  time_fft2_body<TS, TC, MODE, ACC64, L1, L2>(J, (const TC*)J.tw, (const TC*)J.tw4, (const TS*)J.in, (TS*)J.out, J.acc64);
}

// elementwise helpers
template <typename TS>
__global__ void k_cast_from64(long n, const double* __restrict__ a, TS* __restrict__ b) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) st<TS, double>(b, i, a[i]);
}
template <typename TS>
__global__ void k_cast_to64(long n, const TS* __restrict__ a, double* __restrict__ b) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) b[i] = ld<double>(a, i);
}

template <typename TS>
__global__ void k_cast_add64(long n, const TS* __restrict__ a, double* __restrict__ b, const int* __restrict__ state) {
  if (state && done_flag(state)) return;
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) b[i] += ld<double>(a, i);
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// coarse nodal field <- per-axis (1/4,1/2,1/4) at interior coarse nodes, injection on the boundary
template <int D>
__global__ void k_restrict_kappa(int nf, int nc, const double* __restrict__ kf, double* __restrict__ kc) {
  const long nnc = nc + 2, nnf = nf + 2;
  long total = nnc;
  if (D >= 2) total *= nnc;
  if (D >= 3) total *= nnc;
  const long q = long(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= total) return;
  int I[3] = {0, 0, 0};
  long rem = q;
  I[0] = int(rem % nnc); rem /= nnc;
  if (D >= 2) { I[1] = int(rem % nnc); rem /= nnc; }
  if (D >= 3) { I[2] = int(rem); }
  double acc = 0.0;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= D) { lo[a] = hi[a] = 0; continue; }
    const bool bnd = (I[a] == 0 || I[a] == nc + 1);
    lo[a] = bnd ? 0 : -1;
    hi[a] = bnd ? 0 : 1;
  }
  for (int dz = lo[2]; dz <= hi[2]; ++dz)
    for (int dy = lo[1]; dy <= hi[1]; ++dy)
      for (int dx = lo[0]; dx <= hi[0]; ++dx) {
        const int d[3] = {dx, dy, dz};
        double w = 1.0;
        long fi = 0;
        for (int a = D - 1; a >= 0; --a) {
          const bool bnd = (I[a] == 0 || I[a] == nc + 1);
          const double wa = bnd ? 1.0 : (d[a] == 0 ? 0.5 : 0.25);
          w *= wa;
          const int fa = 2 * I[a] + d[a];
          fi = fi * nnf + fa;
        }
        acc += w * kf[fi];
      }
  kc[q] = acc;
}

template <typename TC>
__global__ void k_scale_copy(long n, const double* __restrict__ a, double s, TC* __restrict__ b) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) b[i] = TC(a[i] * s);
}

// ---------------------------------------------------------------------------
// vector helpers of the damping estimate (setup only)
// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator:
// state = seed + (i + 1) * golden gamma, then the output mix; the top 53 bits
// give a value in [-1, 1).
__device__ __forceinline__ double splitmix_pm1(unsigned long long i, unsigned long long seed) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return double(z >> 11) * 0x1.0p-52 - 1.0;
}

#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void k_fill_pm1(long n, unsigned long long seed, double* __restrict__ out) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = splitmix_pm1((unsigned long long)i, seed);
}
#endif

// block partials of a . b over a fixed grid (grid-stride), summed by k_sum_to
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_dot_partial(long n, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ partial) {
  double v = 0.0;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n; i += long(gridDim.x) * kBlock) v += a[i] * b[i];
  const double s = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
#endif

// y = a x + b y  (y is not read when b == 0)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void k_axpby(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
#endif

// b = s * a, widened to float64
template <typename TS>
__global__ void k_cast_scale64(long n, const TS* __restrict__ a, double s, double* __restrict__ b) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) b[i] = s * ld<double>(a, i);
}

// min over slabs s < S and nodes of sum_r coef[s][r] * fields[r][node]  (block partials)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void k_kappa_min(long nnodes, int R, int S, const double* __restrict__ fields,
                            const double* __restrict__ coef, double* __restrict__ partial) {
  __shared__ double red[kBlock];
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double m = 1e300;
  if (i < nnodes) {
    double f[kMaxRank];
    for (int r = 0; r < kMaxRank; ++r) f[r] = r < R ? fields[r * nnodes + i] : 0.0;
    for (int s = 0; s < S; ++s) {
      double k = 0.0;
      for (int r = 0; r < R; ++r) k += coef[s * kMaxRank + r] * f[r];
      m = fmin(m, k);
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
#endif

// ---------------------------------------------------------------------------
// Krylov acceleration (GMRES around the Uzawa sweep), float64 vectors
// ---------------------------------------------------------------------------
// r = g - saddle [p; u] with g = [-f; -f], f_s = tau_s F_s (+ u0 on the first slab)
template <int D>
__global__ void __launch_bounds__(kBlock) k_saddle_resid(Geom g, TimeOp t, const double* __restrict__ taus,
                                                         const double* __restrict__ F,
                                                         const double* __restrict__ u0, const double* __restrict__ p,
                                                         const double* __restrict__ u, double* __restrict__ rp,
                                                         double* __restrict__ ru) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= t.N || i >= g.npts) return;
  int px, py, pz;
  decode<D>(i, g.n, px, py, pz);
  const SlabOp<double> op = load_op<double>(nullptr, t.cA, s, t.R);
  const long o = long(s) * g.npts;
  double dg, offp, offu;
  stencil2<D>(p + o, u + o, i, px, py, pz, g, t.kap, op, t.R, dg, offp, offu);
  const double pc = p[o + i];
  const double uc = u[o + i];
  const double Ap = dg * pc - offp;
  const double Au = dg * uc - offu;
  const double um = s > 0 ? u[o - g.npts + i] : 0.0;
  const double up = s + 1 < t.N ? u[o + g.npts + i] : 0.0;
  const double pp = s + 1 < t.N ? p[o + g.npts + i] : 0.0;
  double f = taus[s] * F[o + i];
  if (s == 0) f += u0[i];
  rp[o + i] = -f - (Ap - (uc - um));
  ru[o + i] = -f + (pc - pp) + (2.0 * uc - um - up) + Au;
}

// block partials of ||f - B u||^2 over a (points, slabs) grid
template <int D>
__global__ void __launch_bounds__(kBlock) k_fmBu_partial(Geom g, TimeOp t, const double* __restrict__ taus,
                                                         const double* __restrict__ F,
                                                         const double* __restrict__ u0, const double* __restrict__ u,
                                                         double* __restrict__ partial) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double v = 0.0;
  if (s < t.N && i < g.npts) {
    int px, py, pz;
    decode<D>(i, g.n, px, py, pz);
    const SlabOp<double> op = load_op<double>(nullptr, t.cA, s, t.R);
    const long o = long(s) * g.npts;
    double dg, off;
    stencil<D, double>(u + o, i, px, py, pz, g, t.kap, op, t.R, dg, off);
    const double uc = u[o + i];
    const double um = s > 0 ? u[o - g.npts + i] : 0.0;
    double f = taus[s] * F[o + i];
    if (s == 0) f += u0[i];
    const double e = f - ((uc - um) + (dg * uc - off));
    v = e * e;
  }
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
}

// out_s = sgn (r_s + d_s - d_{s+1})  (sgn (r + K^T d), d_N := 0), in the storage
// type of the preconditioner's input
template <typename TS>
__global__ void k_kt_add_cast(long npts, int N, const double* __restrict__ r, const double* __restrict__ d,
                              double sgn, TS* __restrict__ out) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  const long n = long(N) * npts;
  if (i >= n) return;
  const double dn = i + npts < n ? d[i + npts] : 0.0;
  st<TS, double>(out, i, sgn * (r[i] + d[i] - dn));
}

constexpr int kDotRows = 8;   // basis vectors per multi-dot launch

// partial[q * gridDim.x + block] = block part of <V_q, w> for q < k (V_q = V + q ld),
// and, when self != 0, row k = block part of <w, w>
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_mdot_partial(long n, const double* __restrict__ V, long ld, int k,
                                                         int self, const double* __restrict__ w,
                                                         double* __restrict__ partial) {
  __shared__ double red[kDotRows + 1][kBlock / 64];
  double acc[kDotRows + 1];
#pragma unroll
  for (int q = 0; q <= kDotRows; ++q) acc[q] = 0.0;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n; i += long(gridDim.x) * kBlock) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < kDotRows; ++q)
      if (q < k) acc[q] += V[q * ld + i] * wi;
    acc[kDotRows] += wi * wi;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q <= kDotRows; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[q][wid] = v;
  }
  __syncthreads();
  const int rows = k + (self ? 1 : 0);
  if (int(threadIdx.x) < rows) {
    const int q = int(threadIdx.x) < k ? int(threadIdx.x) : kDotRows;
    double sum = 0.0;
    for (int w2 = 0; w2 < kBlock / 64; ++w2) sum += red[q][w2];
    partial[long(threadIdx.x) * gridDim.x + blockIdx.x] = sum;
  }
}
#endif

// out[row] = sum of partial[row * count .. row * count + count), one block per row
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_sum_rows(const double* __restrict__ partial, long count,
                                                     double* __restrict__ out) {
  const double* pr = partial + long(blockIdx.x) * count;
  double v = 0.0;
  for (long q = threadIdx.x; q < count; q += kBlock) v += pr[q];
  const double s = block_sum(v);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}
#endif

// w -= sum_{q<k} coef[q] V_q over a fixed grid (grid-stride), with block
// partials of the updated ||w||^2 (summed by k_sum_rows)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_maxpy_norm(long n, double* __restrict__ w, const double* __restrict__ V,
                                                       long ld, int k, const double* __restrict__ coef,
                                                       double* __restrict__ partial) {
  double v = 0.0;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < n; i += long(gridDim.x) * kBlock) {
    double acc = 0.0;
    for (int q0 = 0; q0 < k; q0 += 8) {   // eight independent loads in flight
      double vv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) vv[t] = q0 + t < k ? V[(q0 + t) * ld + i] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (q0 + t < k) acc += coef[q0 + t] * vv[t];
    }
    const double wi = w[i] - acc;
    w[i] = wi;
    v += wi * wi;
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
#endif

// w += sgn * sum_{q<k} coef[q] V_q  (coefficients read from device memory)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void k_maxpy(long n, double* __restrict__ w, const double* __restrict__ V, long ld, int k,
                        const double* __restrict__ coef, double sgn) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int q0 = 0; q0 < k; q0 += 8) {
    double vv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) vv[t] = q0 + t < k ? V[(q0 + t) * ld + i] : 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (q0 + t < k) acc += coef[q0 + t] * vv[t];
  }
  w[i] += sgn * acc;
}
#endif

}  // namespace stp

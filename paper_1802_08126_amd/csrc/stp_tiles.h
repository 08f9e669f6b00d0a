// LDS-tiled stencil kernels: the fused multigrid level kernels and the
// time-global residual kernels.
//
// Every block owns one spatial tile of one slab.  It stages into LDS the
// slab-combined coefficient kappa_s = sum_r c_{s,r} k_r (k_r = kappa_r / 2h^2,
// nodal, incl. boundary) over the tile plus the halo its stencils need, so a
// face weight is kappa_s[i] + kappa_s[nb] and the diagonal is
// sigma_s + sum over the 2d faces.
//
// Node coordinates are 1-based with 0 and n+1 on the boundary; the interior
// vector entry of node j sits at offset j-1 per axis.
//
// The kernels are written to keep the per-point instruction count low (they
// would otherwise be issue-bound rather than HBM-bound): boxes are walked with
// an incremental, division-free iterator, bounds tests are single unsigned
// compares, offsets inside a slab are 32-bit, and the Jacobi divisions use
// the hardware reciprocal refined by Newton steps.
#pragma once
#include "stp_kernels.h"

namespace stp {

template <int D, int EX, int EY, int EZ, int NTH = kBlock>
struct Box {
  static constexpr int threads = NTH;   // threads of the block that walks the box
  static constexpr int X = EX;
  static constexpr int Y = (D >= 2 ? EY : 1);
  static constexpr int Z = (D >= 3 ? EZ : 1);
  static constexpr int size = X * Y * Z;
  __device__ static __forceinline__ int idx(int x, int y, int z) { return (z * Y + y) * X + x; }
};

// Walks the linear positions q = threadIdx.x, threadIdx.x + B::threads, ... of
// a box, keeping (x, y, z) up to date with adds and one conditional subtract
// per axis instead of divisions.
template <typename B>
struct BoxIter {
  static constexpr int DX = B::threads % B::X;
  static constexpr int DR = B::threads / B::X;
  static constexpr int DY = DR % B::Y;
  static constexpr int DZ = DR / B::Y;
  int q, x, y, z;
  __device__ __forceinline__ BoxIter() {
    q = threadIdx.x;
    x = q % B::X;
    const int r = q / B::X;
    y = r % B::Y;
    z = r / B::Y;
  }
  __device__ __forceinline__ bool ok() const { return q < B::size; }
  __device__ __forceinline__ void next() {
    q += B::threads;
    x += DX;
    int cy = 0;
    if (x >= B::X) { x -= B::X; cy = 1; }
    y += DY + cy;
    int cz = 0;
    if (y >= B::Y) { y -= B::Y; cz = 1; }
    z += DZ + cz;
  }
};

template <typename B>
__host__ __device__ constexpr int nit() {
  return (B::size + B::threads - 1) / B::threads;
}

// Fully unrolled walk over a box (compile-time trip count); `continue` in the
// body moves on to the next position.
#define STP_BOX_FOR(B, it)                                                  \
  _Pragma("unroll") for (BoxIter<B> it; it.q < int(threadIdx.x) + nit<B>() * B::threads; it.next()) \
    if (it.ok())

// offsets of the 2d neighbours inside a box (x-, x+, y-, y+, z-, z+)
template <typename B>
__device__ __forceinline__ constexpr int nb_off(int k) {
  return k == 0 ? -1 : k == 1 ? 1 : k == 2 ? -B::X : k == 3 ? B::X : k == 4 ? -B::X * B::Y : B::X * B::Y;
}

__device__ __forceinline__ bool in_range(int j, int lo, int hi) { return unsigned(j - lo) <= unsigned(hi - lo); }

template <int D>
__device__ __forceinline__ bool in_nodes(int jx, int jy, int jz, int n) {
  bool ok = in_range(jx, 0, n + 1);
  if (D >= 2) ok = ok && in_range(jy, 0, n + 1);
  if (D >= 3) ok = ok && in_range(jz, 0, n + 1);
  return ok;
}

template <int D>
__device__ __forceinline__ bool interior(int jx, int jy, int jz, int n) {
  bool ok = in_range(jx, 1, n);
  if (D >= 2) ok = ok && in_range(jy, 1, n);
  if (D >= 3) ok = ok && in_range(jz, 1, n);
  return ok;
}

// node (incl. boundary) -> offset in a nodal field; interior node -> vector offset
template <int D>
__device__ __forceinline__ int node_off(int jx, int jy, int jz, int n) {
  const int nn = n + 2;
  if (D == 1) return jx;
  if (D == 2) return jy * nn + jx;
  return (jz * nn + jy) * nn + jx;
}
template <int D>
__device__ __forceinline__ int vec_off(int jx, int jy, int jz, int n) {
  if (D == 1) return jx - 1;
  if (D == 2) return (jy - 1) * n + (jx - 1);
  return ((jz - 1) * n + (jy - 1)) * n + (jx - 1);
}

// reciprocal: hardware estimate + Newton refinement (float64), hardware (float32)
__device__ __forceinline__ double rcp_fast(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_fast(float d) { return __builtin_amdgcn_rcpf(d); }

// Stage kappa_s over box KB whose origin is node (ox, oy, oz).  All global
// loads of the thread are issued before the first LDS store.
template <int D, typename KB, typename TC>
__device__ __forceinline__ void stage_kappa(TC* sk, const TC* __restrict__ kap, long nnodes, int n, int ox, int oy,
                                            int oz, const SlabOp<TC>& op, int R) {
  constexpr int NI = nit<KB>();
  TC v[NI];
  BoxIter<KB> it;
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    v[k] = 0;
    if (it.ok()) {
      const int jx = ox + it.x, jy = oy + it.y, jz = oz + it.z;
      if (in_nodes<D>(jx, jy, jz, n)) {
        const int o = node_off<D>(jx, jy, jz, n);
        v[k] = op.c[0] * kap[o];
#pragma unroll
        for (int r = 1; r < kMaxRank; ++r)
          if (r < R) v[k] += op.c[r] * kap[r * nnodes + o];
      }
    }
    it.next();
  }
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int q = threadIdx.x + k * KB::threads;
    if (q < KB::size) sk[q] = v[k];
  }
}

// Load a TS vector over box B (origin node (ox, oy, oz)) into registers,
// zero outside the interior.
template <int D, typename B, typename TS, typename TC>
__device__ __forceinline__ void prefetch_box(TC (&v)[nit<B>()], const TS* __restrict__ xs, int n, int ox, int oy,
                                             int oz) {
  BoxIter<B> it;
#pragma unroll
  for (int k = 0; k < nit<B>(); ++k) {
    v[k] = 0;
    if (it.ok()) {
      const int jx = ox + it.x, jy = oy + it.y, jz = oz + it.z;
      if (interior<D>(jx, jy, jz, n)) v[k] = ld<TC>(xs, vec_off<D>(jx, jy, jz, n));
    }
    it.next();
  }
}

// diagonal at x-box position xq; the kappa box is one node larger on each side
template <int D, typename KB, typename TC>
__device__ __forceinline__ TC diag_at_k(const TC* sk, int kq, TC sigma) {
  const TC kc = sk[kq];
  TC d = sigma + TC(2 * D) * kc;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) d += sk[kq + nb_off<KB>(k)];
  return d;
}

template <int D, typename XB, typename KB, typename TC>
__device__ __forceinline__ TC offsum_at(const TC* sk, const TC* sx, int kq, int xq) {
  const TC kc = sk[kq];
  TC o = 0;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) o += (kc + sk[kq + nb_off<KB>(k)]) * sx[xq + nb_off<XB>(k)];
  return o;
}

// fixed-field launches: k_fix staged once per block over box KB (origin ox, oy, oz)
template <int D, typename KB, typename TC>
__device__ __forceinline__ void stage_fixed(TC* sk, const LevelOp& L, long nnodes, int n, int ox, int oy, int oz) {
  const TC* kap = (const TC*)L.kap;
  TC f[kMaxRank];
#pragma unroll
  for (int r = 0; r < kMaxRank; ++r) f[r] = r < L.R ? fixed_coef<TC>(L, r) : TC(0);
  BoxIter<KB> it;
#pragma unroll
  for (int k = 0; k < nit<KB>(); ++k) {
    if (it.ok()) {
      const int jx = ox + it.x, jy = oy + it.y, jz = oz + it.z;
      TC v = 0;
      if (in_nodes<D>(jx, jy, jz, n)) {
        const int o = node_off<D>(jx, jy, jz, n);
        v = f[0] * kap[o];
        for (int r = 1; r < L.R; ++r) v += f[r] * kap[r * nnodes + o];
      }
      sk[it.q] = v;
    }
    it.next();
  }
}

// diagonal sigma + gamma (2d k_c + sum_nb k_nb) of a fixed-field launch
template <int D, typename KB, typename TC>
__device__ __forceinline__ TC diag_fixed(const TC* sk, int kq, TC sigma, TC gamma) {
  const TC kc = sk[kq];
  TC d = TC(2 * D) * kc;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) d += sk[kq + nb_off<KB>(k)];
  return sigma + gamma * d;
}

// face sums 2d k_c + sum_nb k_nb of a fixed field (staged in sk over KB) at
// every position of box XB (KB one node larger on each side)
template <int D, typename XB, typename KB, typename TC>
__device__ __forceinline__ void stage_facesum(TC* sd, const TC* sk);

// kappa-box position of x-box position (x, y, z) when KB is one node larger
template <int D, typename KB>
__device__ __forceinline__ int kpos(int x, int y, int z) {
  return KB::idx(x + 1, D >= 2 ? y + 1 : 0, D >= 3 ? z + 1 : 0);
}

template <int D, typename XB, typename KB, typename TC>
__device__ __forceinline__ void stage_facesum(TC* sd, const TC* sk) {
  BoxIter<XB> it;
#pragma unroll
  for (int k = 0; k < nit<XB>(); ++k) {
    if (it.ok()) {
      const int kq = kpos<D, KB>(it.x, it.y, it.z);
      TC d = TC(2 * D) * sk[kq];
#pragma unroll
      for (int j = 0; j < 2 * D; ++j) d += sk[kq + nb_off<KB>(j)];
      sd[it.q] = d;
    }
    it.next();
  }
}

// ---------------------------------------------------------------------------
// tile shapes
// ---------------------------------------------------------------------------
template <int D> struct DownTile;
template <> struct DownTile<1> { static constexpr int X = 256, Y = 1, Z = 1; };
template <> struct DownTile<2> { static constexpr int X = 32, Y = 8, Z = 1; };
template <> struct DownTile<3> { static constexpr int X = 8, Y = 4, Z = 4; };

template <int D> struct UpTile;
template <> struct UpTile<1> { static constexpr int X = 512, Y = 1, Z = 1; };
template <> struct UpTile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct UpTile<3> { static constexpr int X = 32, Y = 4, Z = 4; };

// tiles of the two time-global residuals: in 3-D twice as tall in y as the
// up-sweep's, with a block of 512 threads so each thread still keeps two points
// in registers: a tile's operand halo is mostly read from HBM again (neighbouring
// tiles march through their slab runs out of step), and 34 x 10 x 6 nodes per
// 32 x 8 x 4 tile are 1.99 reads per point against 2.39 for 32 x 4 x 4.  On
// 255^3 x 64 (float32) a1 / a3 took 7.79 / 7.96 ms against 8.01 / 8.21; 32 x 8 x 8
// with 1024 threads (one block per CU) 7.77 / 8.36, and 32 x 8 x 4 with 256
// threads (four points per thread, fewer waves) 7.94 / 9.56.
template <int D> struct ResidTile : UpTile<D> { static constexpr int threads = kBlock; };
template <> struct ResidTile<3> { static constexpr int X = 32, Y = 8, Z = 4, threads = 512; };
// the middle operator of the H-blocks (and the operator after the first of
// several H cycles): the residuals' tile shape, for the same reason
template <int D> struct MidTile : ResidTile<D> {};

template <int D, typename T>
__host__ __device__ inline long tiles_for(int n) {
  long t = (n + T::X - 1) / T::X;
  if (D >= 2) t *= (n + T::Y - 1) / T::Y;
  if (D >= 3) t *= (n + T::Z - 1) / T::Z;
  return t;
}

// 3-D tile order: x fastest, then bricks of kBrickY x kBrickZ tiles in (y, z),
// y fastest inside a brick, so the tiles a few hundred blocks in flight on one
// XCD cover neighbours in z as well as in y and share their halos in its L2
// (row-major order puts the z-neighbours a whole tile plane apart).  On 255^3 x
// 64 the residuals took 4-5 % less time (float32 a1 8.40 -> 8.03 ms).
constexpr bool kTileBricks = true;
constexpr int kBrickY = 4, kBrickZ = 8;

template <int D, typename T>
__device__ __forceinline__ void tile_origin(int n, int tile, int& tx, int& ty, int& tz) {
  const int ntx = (n + T::X - 1) / T::X;
  const int nty = D >= 2 ? (n + T::Y - 1) / T::Y : 1;
  int t = tile;
  tx = t % ntx;
  t /= ntx;
  if (D == 3 && kTileBricks) {
    const int ntz = (n + T::Z - 1) / T::Z;
    const int zb = t / (nty * kBrickZ), rz0 = zb * kBrickZ, bz = min(kBrickZ, ntz - rz0);
    const int q = t - zb * nty * kBrickZ;
    const int yb = q / (kBrickY * bz), ry0 = yb * kBrickY, by = min(kBrickY, nty - ry0);
    const int q2 = q - yb * kBrickY * bz;
    ty = ry0 + q2 % by;
    tz = rz0 + q2 / by;
    return;
  }
  ty = D >= 2 ? t % nty : 0;
  tz = D >= 3 ? t / nty : 0;
}

// ---------------------------------------------------------------------------
// slab pipelining
//
// A block processes one spatial tile for a run of consecutive slabs
// [s0, s0 + sb): the slab-independent coefficient fields of the tile are
// loaded into registers once, and the next slab's vectors are prefetched into
// registers while the current slab is computed from LDS, so global-memory
// latency overlaps with work.  blockIdx.y (+ gridDim.y * blockIdx.z) numbers
// the slab runs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rank_bound_ok(int r, int R) { return r < R; }

// raw fields r < R over box KB (origin node ox, oy, oz); zero elsewhere
template <int D, typename KB, typename TC, int RM>
__device__ __forceinline__ void load_kraw(TC (&kr)[nit<KB>()][RM], const TC* __restrict__ kap, long nnodes, int R,
                                          int n, int ox, int oy, int oz) {
  BoxIter<KB> it;
#pragma unroll
  for (int k = 0; k < nit<KB>(); ++k) {
#pragma unroll
    for (int r = 0; r < RM; ++r) kr[k][r] = 0;
    if (it.ok()) {
      const int jx = ox + it.x, jy = oy + it.y, jz = oz + it.z;
      if (in_nodes<D>(jx, jy, jz, n)) {
        const int o = node_off<D>(jx, jy, jz, n);
#pragma unroll
        for (int r = 0; r < RM; ++r)
          if (r < R) kr[k][r] = kap[r * nnodes + o];
      }
    }
    it.next();
  }
}

template <typename KB, typename TC, int RM>
__device__ __forceinline__ void write_kappa(TC* sk, const TC (&kr)[nit<KB>()][RM], const SlabOp<TC>& op) {
#pragma unroll
  for (int k = 0; k < nit<KB>(); ++k) {
    const int q = threadIdx.x + k * KB::threads;
    if (q < KB::size) {
      TC v = op.c[0] * kr[k][0];
#pragma unroll
      for (int r = 1; r < RM; ++r) v += op.c[r] * kr[k][r];
      sk[q] = v;
    }
  }
}

template <typename B, typename TC>
__device__ __forceinline__ void write_box(TC* sx, const TC (&v)[nit<B>()]) {
#pragma unroll
  for (int k = 0; k < nit<B>(); ++k) {
    const int q = threadIdx.x + k * B::threads;
    if (q < B::size) sx[q] = v[k];
  }
}

template <int N_>
struct Regs {
  template <typename TC>
  __device__ static __forceinline__ void copy(TC (&dst)[N_], const TC (&src)[N_]) {
#pragma unroll
    for (int k = 0; k < N_; ++k) dst[k] = src[k];
  }
};

// the block's job (copied to scalar registers), tile index and slab run [s0, s1)
template <typename J>
__device__ __forceinline__ J job_tile_run(const J* __restrict__ jobs, int njobs, int S, int& tile, int& s0, int& s1) {
  const J job = to_global(jobs[find_job(jobs, njobs)]);
  const int lb = int(block_id() - job.block0);
  tile = lb % job.tiles;
  s0 = (lb / job.tiles) * job.sb;
  s1 = min(S, s0 + job.sb);
  return job;
}

// residual kernels: one job per problem
struct ResidJob {
  long block0;
  int tiles;
  int sb;
  Geom g;
  TimeOp t;
  const double* taus;   // N step lengths tau_n
  const double* u;
  const double* p;
  const double* F;
  const double* u0;
  void* r;
  double* partial;      // one entry per block of the job
  const int* state;
};

__device__ __forceinline__ ResidJob to_global(ResidJob j) {
  j.t.kap = gmem(j.t.kap);
  j.t.cA = gmem(j.t.cA);
  j.taus = gmem(j.taus);
  j.u = gmem(j.u);
  j.p = gmem(j.p);
  j.F = gmem(j.F);
  j.u0 = gmem(j.u0);
  j.r = gmem(j.r);
  j.partial = gmem(j.partial);
  j.state = gmem(j.state);
  return j;
}

// ---------------------------------------------------------------------------
// multigrid: pre-smooth from zero, residual and full-weighting restriction
//   x1 = omega D^{-1} b,  r = b - L x1 = (1 - omega) b + sum_nb w x1_nb,  bc = R r
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC, int RM, bool FIX>
__device__ __forceinline__ void mg_down_body(const TileJob& J, int tile, int s0, int s1, TC omega,
                                             const TS* __restrict__ b, TS* __restrict__ bc) {
  using T = DownTile<D>;
  using KB = Box<D, 2 * T::X + 5, 2 * T::Y + 5, 2 * T::Z + 5>;
  using XB = Box<D, 2 * T::X + 3, 2 * T::Y + 3, 2 * T::Z + 3>;
  using RB = Box<D, 2 * T::X + 1, 2 * T::Y + 1, 2 * T::Z + 1>;
  using CB = Box<D, T::X, T::Y, T::Z>;
  // the residual tile is stored split by the parity of x (rows of RE even and
  // RO odd positions), so the restriction's three x-taps of consecutive coarse
  // nodes are unit-stride LDS reads instead of stride 2 (bank conflicts)
  constexpr int RE = T::X + 1, RO = T::X;
  constexpr int RROWS = RB::Y * RB::Z;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[XB::size];
  __shared__ TC sre[RROWS * RE];
  __shared__ TC sro[RROWS * RO];
  // fixed field: the slab-independent face sum 2d k_c + sum_nb k_nb of every
  // x1-box node, so a slab's diagonal is sigma + gamma * sd (one LDS read)
  __shared__ TC sd[FIX ? XB::size : 1];
  const LevelOp L = J.op;
  s1 = min(s1, L.S);
  if (s0 >= s1) return;
  const Geom gf = J.gf, gc = J.gc;
  const int nf = gf.n, nc = gc.n;
  int tx, ty, tz;
  tile_origin<D, T>(nc, tile, tx, ty, tz);
  // first coarse node of the tile (1-based); the fine node of coarse I is 2I
  const int Ix = tx * T::X + 1, Iy = D >= 2 ? ty * T::Y + 1 : 1, Iz = D >= 3 ? tz * T::Z + 1 : 1;
  const int rx = 2 * Ix - 1, ry = D >= 2 ? 2 * Iy - 1 : 1, rz = D >= 3 ? 2 * Iz - 1 : 1;   // r-box origin
  const int xx = rx - 1, xy = D >= 2 ? ry - 1 : 1, xz = D >= 3 ? rz - 1 : 1;                // x1-box origin
  TC kr[FIX ? 1 : nit<KB>()][FIX ? 1 : RM];
  if constexpr (FIX) {
    stage_fixed<D, KB, TC>(sk, L, gf.nnodes, nf, xx - 1, D >= 2 ? xy - 1 : 1, D >= 3 ? xz - 1 : 1);
    __syncthreads();
    stage_facesum<D, XB, KB, TC>(sd, sk);
    __syncthreads();
  } else {
    load_kraw<D, KB, TC, RM>(kr, (const TC*)L.kap, gf.nnodes, L.R, nf, xx - 1, D >= 2 ? xy - 1 : 1,
                             D >= 3 ? xz - 1 : 1);
  }
  TC bn[nit<XB>()];
  prefetch_box<D, XB, TS, TC>(bn, b + long(s0) * gf.npts, nf, xx, xy, xz);
  const TC one_m_omega = TC(1) - omega;
  for (int s = s0; s < s1; ++s) {
    TC bcur[nit<XB>()];
    Regs<nit<XB>()>::copy(bcur, bn);
    if (s + 1 < s1) prefetch_box<D, XB, TS, TC>(bn, b + long(s + 1) * gf.npts, nf, xx, xy, xz);
    const SlabOp<TC> op = level_op<TC>(L, s);
    const TC gamma = FIX ? slab_scale<TC>(L, s) : TC(1);
    if constexpr (!FIX) {
      write_kappa<KB, TC, RM>(sk, kr, op);
      __syncthreads();
    }   // FIX: the field is staged once; every phase ends in a barrier
    {
      BoxIter<XB> it;
#pragma unroll
      for (int k = 0; k < nit<XB>(); ++k) {
        if (it.ok()) {
          const int jx = xx + it.x, jy = xy + it.y, jz = xz + it.z;
          TC v = 0;
          if (interior<D>(jx, jy, jz, nf))
            v = omega * bcur[k] *
                rcp_fast(FIX ? op.sigma + gamma * sd[FIX ? it.q : 0]
                             : diag_at_k<D, KB, TC>(sk, kpos<D, KB>(it.x, it.y, it.z), op.sigma));
          sx[it.q] = v;
        }
        it.next();
      }
    }
    __syncthreads();
    {
      // the r-box is the interior of the x1-box (r-box position = x1-box position - 1);
      // walking the x1-box with the same thread mapping keeps b in registers.  Nodes
      // outside the domain have b = x1 = 0 (their r is never restricted).
      BoxIter<XB> it;
#pragma unroll
      for (int k = 0; k < nit<XB>(); ++k) {
        if (it.ok()) {
          bool inr = in_range(it.x, 1, XB::X - 2);
          if (D >= 2) inr = inr && in_range(it.y, 1, XB::Y - 2);
          if (D >= 3) inr = inr && in_range(it.z, 1, XB::Z - 2);
          if (inr) {
            const int px = it.x - 1;
            const int row = (D >= 2 ? it.y - 1 : 0) + (D >= 3 ? (it.z - 1) * RB::Y : 0);
            const TC off = offsum_at<D, XB, KB, TC>(sk, sx, kpos<D, KB>(it.x, it.y, it.z), it.q);
            const TC rv = one_m_omega * bcur[k] + (FIX ? gamma * off : off);
            if (px & 1) sro[row * RO + (px >> 1)] = rv;
            else sre[row * RE + (px >> 1)] = rv;
          }
        }
        it.next();
      }
    }
    __syncthreads();
    TS* bcs = bc + long(s) * gc.npts;
    STP_BOX_FOR(CB, it) {
      const int Jx = Ix + it.x, Jy = Iy + it.y, Jz = Iz + it.z;
      if (!interior<D>(Jx, Jy, Jz, nc)) continue;
      // fine node 2J sits at r-box position 2x+1 per axis: x-taps 2x (even row
      // entry x), 2x+1 (odd entry x) and 2x+2 (even entry x+1)
      const int r0 = (D >= 2 ? 2 * it.y + 1 : 0) + (D >= 3 ? (2 * it.z + 1) * RB::Y : 0);
      TC acc = 0;
#pragma unroll
      for (int dz = (D >= 3 ? -1 : 0); dz <= (D >= 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
          TC w = 1;
          if (D >= 2) w *= (dy == 0 ? TC(0.5) : TC(0.25));
          if (D >= 3) w *= (dz == 0 ? TC(0.5) : TC(0.25));
          const int row = r0 + dz * RB::Y + dy;
          acc += w * (TC(0.25) * sre[row * RE + it.x] + TC(0.5) * sro[row * RO + it.x] +
                      TC(0.25) * sre[row * RE + it.x + 1]);
        }
      st<TS, TC>(bcs, vec_off<D>(Jx, Jy, Jz, nc), acc);
    }
    // the next slab writes sk only after every thread has passed the barrier
    // that ends its x1 phase, and sr only after two more barriers
  }
}

// Launch variants V: 0 = every job per-slab coefficients, 1 = every job a fixed
// field, 2 = mixed (each job runs the body of its own mode, so a problem's
// arithmetic never depends on the batch it is in)
__device__ __forceinline__ bool job_fixed(int V, int cmode) { return V == 1 || (V == 2 && cmode != CM_SLAB); }

template <int D, typename TS, typename TC, int RM, int V>
__global__ void __launch_bounds__(kBlock) k_mg_down(const TileJob* __restrict__ jobs, int njobs, TC omega) {
  int tile, s0, s1;
  const TileJob J = job_tile_run(jobs, njobs, 1 << 30, tile, s0, s1);
  if (J.state && done_flag(J.state)) return;
  if (job_fixed(V, J.op.cmode)) mg_down_body<D, TS, TC, RM, true>(J, tile, s0, s1, omega, (const TS*)J.b, (TS*)J.out);
  else mg_down_body<D, TS, TC, RM, false>(J, tile, s0, s1, omega, (const TS*)J.b, (TS*)J.out);
}

// ---------------------------------------------------------------------------
// multigrid: coarse correction and post-smoothing
//   x2 = omega D^{-1} b + P e,   x = (1 - omega) x2 + omega D^{-1} (b + sum_nb w x2_nb)
// epilogue: store x (TS) or add it into a float64 vector
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC, int RM, int EPI, bool FIX>
__device__ __forceinline__ void mg_up_body(const TileJob& J, int tile, int s0, int s1, TC omega,
                                           const TS* __restrict__ b, const TS* __restrict__ e, TS* __restrict__ out,
                                           double* __restrict__ acc64) {
  using T = UpTile<D>;
  using KB = Box<D, T::X + 4, T::Y + 4, T::Z + 4>;
  using XB = Box<D, T::X + 2, T::Y + 2, T::Z + 2>;
  using EB = Box<D, T::X / 2 + 2, T::Y / 2 + 2, T::Z / 2 + 2>;
  using TB = Box<D, T::X, T::Y, T::Z>;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[XB::size];
  __shared__ TC sb_[XB::size];
  __shared__ TC se[EB::size];
  __shared__ TC sd[FIX ? XB::size : 1];   // fixed field: face sums of the x2-box nodes
  const LevelOp L = J.op;
  s1 = min(s1, L.S);
  if (s0 >= s1) return;
  const Geom gf = J.gf, gc = J.gc;
  const int nf = gf.n, nc = gc.n;
  int tx, ty, tz;
  tile_origin<D, T>(nf, tile, tx, ty, tz);
  const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
  const int xx = jx0 - 1, xy = D >= 2 ? jy0 - 1 : 1, xz = D >= 3 ? jz0 - 1 : 1;   // x2-box origin
  const int ex = xx / 2, ey = D >= 2 ? xy / 2 : 1, ez = D >= 3 ? xz / 2 : 1;      // first coarse node
  TC kr[FIX ? 1 : nit<KB>()][FIX ? 1 : RM];
  if constexpr (FIX) {
    stage_fixed<D, KB, TC>(sk, L, gf.nnodes, nf, xx - 1, D >= 2 ? xy - 1 : 1, D >= 3 ? xz - 1 : 1);
    __syncthreads();
    stage_facesum<D, XB, KB, TC>(sd, sk);   // read after the first slab's barrier
  } else {
    load_kraw<D, KB, TC, RM>(kr, (const TC*)L.kap, gf.nnodes, L.R, nf, xx - 1, D >= 2 ? xy - 1 : 1,
                             D >= 3 ? xz - 1 : 1);
  }
  TC bn[nit<XB>()];
  TC en[nit<EB>()];
  prefetch_box<D, XB, TS, TC>(bn, b + long(s0) * gf.npts, nf, xx, xy, xz);
  prefetch_box<D, EB, TS, TC>(en, e + long(s0) * gc.npts, nc, ex, ey, ez);
  const TC one_m_omega = TC(1) - omega;
  for (int s = s0; s < s1; ++s) {
    TC bcur[nit<XB>()];
    Regs<nit<XB>()>::copy(bcur, bn);
    const SlabOp<TC> op = level_op<TC>(L, s);
    const TC gamma = FIX ? slab_scale<TC>(L, s) : TC(1);
    if constexpr (!FIX) write_kappa<KB, TC, RM>(sk, kr, op);
    write_box<EB, TC>(se, en);
    if (s + 1 < s1) {
      prefetch_box<D, XB, TS, TC>(bn, b + long(s + 1) * gf.npts, nf, xx, xy, xz);
      prefetch_box<D, EB, TS, TC>(en, e + long(s + 1) * gc.npts, nc, ex, ey, ez);
    }
    __syncthreads();
    {
      BoxIter<XB> it;
#pragma unroll
      for (int k = 0; k < nit<XB>(); ++k) {
        if (it.ok()) {
          const int jx = xx + it.x, jy = xy + it.y, jz = xz + it.z;
          TC v = 0;
          if (interior<D>(jx, jy, jz, nf)) {
            const TC wd =
                omega * rcp_fast(FIX ? op.sigma + gamma * sd[FIX ? it.q : 0]
                                     : diag_at_k<D, KB, TC>(sk, kpos<D, KB>(it.x, it.y, it.z), op.sigma));
            // multilinear interpolation from coarse nodes floor(j/2) and, for odd j, floor(j/2)+1
            const int lx = (jx >> 1) - ex, ly = D >= 2 ? (jy >> 1) - ey : 0, lz = D >= 3 ? (jz >> 1) - ez : 0;
            const int ox = jx & 1, oy = D >= 2 ? (jy & 1) : 0, oz = D >= 3 ? (jz & 1) : 0;
            const int e0 = EB::idx(lx, ly, lz);
            auto px = [&](int base) -> TC { return ox ? TC(0.5) * (se[base] + se[base + 1]) : se[base]; };
            TC pe;
            if (D == 1) {
              pe = px(e0);
            } else if (D == 2) {
              pe = oy ? TC(0.5) * (px(e0) + px(e0 + EB::X)) : px(e0);
            } else {
              auto pxy = [&](int base) -> TC { return oy ? TC(0.5) * (px(base) + px(base + EB::X)) : px(base); };
              pe = oz ? TC(0.5) * (pxy(e0) + pxy(e0 + EB::X * EB::Y)) : pxy(e0);
            }
            v = wd * bcur[k] + pe;
          }
          sx[it.q] = v;
          sb_[it.q] = bcur[k];
        }
        it.next();
      }
    }
    __syncthreads();
    TS* os = out ? out + long(s) * gf.npts : nullptr;
    double* as = acc64 ? acc64 + long(s) * gf.npts : nullptr;
    STP_BOX_FOR(TB, it) {
      const int jx = jx0 + it.x, jy = jy0 + it.y, jz = jz0 + it.z;
      if (!interior<D>(jx, jy, jz, nf)) continue;
      const int ax = it.x + 1, ay = D >= 2 ? it.y + 1 : 0, az = D >= 3 ? it.z + 1 : 0;
      const int xq = XB::idx(ax, ay, az);
      const int kq = kpos<D, KB>(ax, ay, az);
      TC off = offsum_at<D, XB, KB, TC>(sk, sx, kq, xq);
      if (FIX) off *= gamma;
      const TC wd = omega * rcp_fast(FIX ? op.sigma + gamma * sd[FIX ? xq : 0]
                                         : diag_at_k<D, KB, TC>(sk, kq, op.sigma));
      const TC v = one_m_omega * sx[xq] + wd * (sb_[xq] + off);
      const int vo = vec_off<D>(jx, jy, jz, nf);
      if (EPI == EPI_STORE) st<TS, TC>(os, vo, J.addout ? ld<TC>(os, vo) + v : v);
      else as[vo] += double(v);
    }
    __syncthreads();   // sk and se are rewritten for the next slab
  }
}

template <int D, typename TS, typename TC, int RM, int EPI, int V>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RM <= 2 ? 4 : 3)))
k_mg_up(const TileJob* __restrict__ jobs, int njobs, TC omega) {
  int tile, s0, s1;
  const TileJob J = job_tile_run(jobs, njobs, 1 << 30, tile, s0, s1);
  if (J.state && done_flag(J.state)) return;
  if (job_fixed(V, J.op.cmode))
    mg_up_body<D, TS, TC, RM, EPI, true>(J, tile, s0, s1, omega, (const TS*)J.b, (const TS*)J.e, (TS*)J.out,
                                         J.acc64);
  else
    mg_up_body<D, TS, TC, RM, EPI, false>(J, tile, s0, s1, omega, (const TS*)J.b, (const TS*)J.e, (TS*)J.out,
                                          J.acc64);
}

// ---------------------------------------------------------------------------
// fused coarse levels: one block per slab runs the whole V-cycle below (and
// including) the fused top level in LDS -- Jacobi from zero, residual and
// full-weighting restriction on the way down, the exact solve on the
// one-node level, multilinear prolongation and the post-sweep on the way up,
// with the formulas of k_mg_down / k_mg_up / k_coarsest.  Every level keeps
// four node-layout arrays ((n+2)^d, boundary nodes zero): the slab-combined
// scaled coefficient, b, the pre-smoothed iterate x, and y (the residual on the
// way down, the level's result on the way up).
// ---------------------------------------------------------------------------
constexpr int kMaxFuse = 9;

struct FuseJob {
  long block0;
  int S;                        // slabs; one block each
  int nlev;                     // fused levels, top first; the last has one node
  int n[kMaxFuse];              // interior nodes per axis
  const void* kap[kMaxFuse];    // scaled fields of each level (TC, R x (n+2)^d)
  LevelOp op;                   // slab rows (op.kap unused)
  const void* b;                // top-level right-hand side (TS)
  void* out;                    // top-level result (TS), or
  double* acc64;                // float64 accumulation target
  const int* state;
  int addout;                   // EPI_STORE: 1 adds the result into out
};

__device__ __forceinline__ FuseJob to_global(FuseJob j) {
  for (int l = 0; l < kMaxFuse; ++l) j.kap[l] = gmem(j.kap[l]);
  j.op = to_global(j.op);
  j.b = gmem(j.b);
  j.out = gmem(j.out);
  j.acc64 = gmem(j.acc64);
  j.state = gmem(j.state);
  return j;
}

template <int D>
__host__ __device__ __forceinline__ long fuse_nodes(int n) {
  const long m = n + 2;
  return D == 1 ? m : (D == 2 ? m * m : m * m * m);
}

// node index of interior point q (0 <= q < n^d), coordinates 1..n
template <int D>
__device__ __forceinline__ int fuse_node_of(int q, int n, int& x, int& y, int& z) {
  const int m = n + 2;
  x = q % n + 1;
  y = D >= 2 ? (q / n) % n + 1 : 0;
  z = D >= 3 ? q / (n * n) + 1 : 0;
  return D == 1 ? x : (D == 2 ? y * m + x : (z * m + y) * m + x);
}

template <int D>
__device__ __forceinline__ int fuse_count(int n) { return D == 1 ? n : (D == 2 ? n * n : n * n * n); }

// Level arrays live at integer offsets of one LDS array (level l: coefficient,
// b, x, y at off(l) + {0, 1, 2, 3} (n_l+2)^d); per-level sizes and fields are
// read from the job table (uniform scalar loads), so nothing is indexed
// dynamically in registers.
template <int D, typename TS, typename TC, int RM, int EPI>
__device__ __forceinline__ void mg_fused_body(const FuseJob* __restrict__ jp, const FuseJob& J, int s, TC omega,
                                              const TS* __restrict__ bin, TS* __restrict__ out,
                                              double* __restrict__ acc64) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* const lds = reinterpret_cast<TC*>(smem_raw);
  const int L = J.nlev;
  auto nodes = [](int n) -> int { const int m = n + 2; return D == 1 ? m : (D == 2 ? m * m : m * m * m); };
  auto loff = [&](int l) -> int {
    int o = 0;
    for (int k = 0; k < l; ++k) o += 4 * nodes(jp->n[k]);
    return o;
  };
  const SlabOp<TC> op = level_op<TC>(J.op, s);
  const int t = threadIdx.x;
  const int nt = blockDim.x;   // 256, 512 or 1024 threads (a schedule choice)
  // coefficients of this slab on every level; zero b, x, y (boundary nodes stay zero)
  {
    int o = 0;
    for (int l = 0; l < L; ++l) {
      const int nn = nodes(jp->n[l]);
      const TC* kl = gmem((const TC*)jp->kap[l]);
      for (int q = t; q < nn; q += nt) {
        TC v = op.c[0] * kl[q];
#pragma unroll
        for (int r = 1; r < RM; ++r)
          if (r < J.op.R) v += op.c[r] * kl[long(r) * nn + q];
        lds[o + q] = v;
      }
      for (int q = t; q < 3 * nn; q += nt) lds[o + nn + q] = TC(0);
      o += 4 * nn;
    }
  }
  __syncthreads();
  {
    const int n = J.n[0];
    const int cnt = fuse_count<D>(n);
    const int ob = nodes(n);   // b of level 0
    const TS* bs = bin + long(s) * cnt;
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      lds[ob + fuse_node_of<D>(q, n, x, y, z)] = ld<TC>(bs, q);
    }
  }
  __syncthreads();
  // stencil pieces at node i of the level whose coefficient starts at ok
  auto diag = [&](int ok, int i, int sy, int sz) -> TC {
    const TC kc = lds[ok + i];
    TC d = op.sigma + TC(2 * D) * kc + lds[ok + i - 1] + lds[ok + i + 1];
    if (D >= 2) d += lds[ok + i - sy] + lds[ok + i + sy];
    if (D >= 3) d += lds[ok + i - sz] + lds[ok + i + sz];
    return d;
  };
  auto offsum = [&](int ok, int ov, int i, int sy, int sz) -> TC {
    const TC kc = lds[ok + i];
    TC o = (kc + lds[ok + i - 1]) * lds[ov + i - 1] + (kc + lds[ok + i + 1]) * lds[ov + i + 1];
    if (D >= 2) o += (kc + lds[ok + i - sy]) * lds[ov + i - sy] + (kc + lds[ok + i + sy]) * lds[ov + i + sy];
    if (D >= 3) o += (kc + lds[ok + i - sz]) * lds[ov + i - sz] + (kc + lds[ok + i + sz]) * lds[ov + i + sz];
    return o;
  };
  const TC one_m_omega = TC(1) - omega;
  // down: x = omega D^-1 b, y = b - L x, b_{l+1} = R y
  int o = 0;
  for (int l = 0; l + 1 < L; ++l) {
    const int n = jp->n[l], m = n + 2, sy = m, sz = m * m, nn = nodes(n);
    const int ok = o, obl = o + nn, ox = o + 2 * nn, oy = o + 3 * nn;
    const int cnt = fuse_count<D>(n);
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const int i = fuse_node_of<D>(q, n, x, y, z);
      lds[ox + i] = omega * lds[obl + i] * rcp_fast(diag(ok, i, sy, sz));
    }
    __syncthreads();
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const int i = fuse_node_of<D>(q, n, x, y, z);
      lds[oy + i] = one_m_omega * lds[obl + i] + offsum(ok, ox, i, sy, sz);
    }
    __syncthreads();
    const int nc = jp->n[l + 1];
    const int obc = o + 4 * nn + nodes(nc);   // b of level l + 1
    const int cntc = fuse_count<D>(nc);
    for (int q = t; q < cntc; q += nt) {
      int X, Y, Z;
      const int ic = fuse_node_of<D>(q, nc, X, Y, Z);
      const int c = D == 1 ? 2 * X : (D == 2 ? (2 * Y) * m + 2 * X : ((2 * Z) * m + 2 * Y) * m + 2 * X);
      TC acc = 0;
#pragma unroll
      for (int dz = (D >= 3 ? -1 : 0); dz <= (D >= 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
          TC w = 1;
          if (D >= 2) w *= (dy == 0 ? TC(0.5) : TC(0.25));
          if (D >= 3) w *= (dz == 0 ? TC(0.5) : TC(0.25));
          const int row = oy + c + dz * sz + dy * sy;
          acc += w * (TC(0.25) * lds[row - 1] + TC(0.5) * lds[row] + TC(0.25) * lds[row + 1]);
        }
      lds[obc + ic] = acc;
    }
    __syncthreads();
    o += 4 * nn;
  }
  // the one-node level: exact solve into y
  {
    const int n = jp->n[L - 1], m = n + 2, nn = nodes(n);
    const int cnt = fuse_count<D>(n);
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const int i = fuse_node_of<D>(q, n, x, y, z);
      lds[o + 3 * nn + i] = lds[o + nn + i] / diag(o, i, m, m * m);
    }
    __syncthreads();
  }
  // up: x += P y_{l+1}; y = (1 - omega) x + omega D^-1 (b + offsum(x))
  for (int l = L - 2; l >= 0; --l) {
    const int n = jp->n[l], m = n + 2, sy = m, sz = m * m, nn = nodes(n);
    const int ol = loff(l);
    const int ok = ol, obl = ol + nn, ox = ol + 2 * nn, oy = ol + 3 * nn;
    const int nc = jp->n[l + 1], mc = nc + 2;
    const int oe = ol + 4 * nn + 3 * nodes(nc);   // y of level l + 1
    const int cnt = fuse_count<D>(n);
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const int i = fuse_node_of<D>(q, n, x, y, z);
      const int e0 = oe + (D == 1 ? (x >> 1)
                           : (D == 2 ? (y >> 1) * mc + (x >> 1) : ((z >> 1) * mc + (y >> 1)) * mc + (x >> 1)));
      const int ox1 = x & 1, oy1 = D >= 2 ? (y & 1) : 0, oz1 = D >= 3 ? (z & 1) : 0;
      auto px = [&](int bq) -> TC { return ox1 ? TC(0.5) * (lds[bq] + lds[bq + 1]) : lds[bq]; };
      TC pe;
      if (D == 1) {
        pe = px(e0);
      } else if (D == 2) {
        pe = oy1 ? TC(0.5) * (px(e0) + px(e0 + mc)) : px(e0);
      } else {
        auto pxy = [&](int bq) -> TC { return oy1 ? TC(0.5) * (px(bq) + px(bq + mc)) : px(bq); };
        pe = oz1 ? TC(0.5) * (pxy(e0) + pxy(e0 + mc * mc)) : pxy(e0);
      }
      lds[ox + i] += pe;
    }
    __syncthreads();
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const int i = fuse_node_of<D>(q, n, x, y, z);
      const TC wd = omega * rcp_fast(diag(ok, i, sy, sz));
      lds[oy + i] = one_m_omega * lds[ox + i] + wd * (lds[obl + i] + offsum(ok, ox, i, sy, sz));
    }
    __syncthreads();
  }
  // top-level result (y of level 0)
  {
    const int n = J.n[0];
    const int cnt = fuse_count<D>(n);
    const int oy = 3 * nodes(n);
    const long ob = long(s) * cnt;
    for (int q = t; q < cnt; q += nt) {
      int x, y, z;
      const TC v = lds[oy + fuse_node_of<D>(q, n, x, y, z)];
      if (EPI == EPI_STORE) st<TS, TC>(out, ob + q, J.addout ? ld<TC>(out, ob + q) + v : v);
      else acc64[ob + q] += double(v);
    }
  }
}

constexpr int kFuseMaxBlock = 1024;

template <int D, typename TS, typename TC, int RM, int EPI>
__global__ void __launch_bounds__(kFuseMaxBlock) k_mg_fused(const FuseJob* __restrict__ jobs, int njobs, TC omega) {
  const int jx = find_job(jobs, njobs);
  const FuseJob J = to_global(jobs[jx]);
  if (J.state && done_flag(J.state)) return;
  const int s = int(block_id() - J.block0);
  if (s >= J.S) return;
  mg_fused_body<D, TS, TC, RM, EPI>(jobs + jx, J, s, omega, (const TS*)J.b, (TS*)J.out, J.acc64);
}

// ---------------------------------------------------------------------------
// y = L x (tile version): the middle reference operator of the H-blocks, whose
// coefficients are the same for every slab; with addout < 0 the step between
// two V-cycles of one application, b -= L x, and with acc_ts / acc64 also
// o += x (H cycles) or p += x (A-tilde cycles, float64)
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC, int RM, bool FIX>
__device__ __forceinline__ void apply_tile_body(const TileJob& J, int tile, int s0, int s1, const TS* __restrict__ xv,
                                                TS* __restrict__ yv) {
  using T = MidTile<D>;
  using KB = Box<D, T::X + 2, T::Y + 2, T::Z + 2, T::threads>;
  using TB = Box<D, T::X, T::Y, T::Z, T::threads>;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[KB::size];
  const LevelOp L = J.op;
  TS* const acc = (TS*)J.acc_ts;
  s1 = min(s1, L.S);
  if (s0 >= s1) return;
  const Geom g = J.gf;
  const int n = g.n;
  int tx, ty, tz;
  tile_origin<D, T>(n, tile, tx, ty, tz);
  const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
  const int ox = jx0 - 1, oy = D >= 2 ? jy0 - 1 : 1, oz = D >= 3 ? jz0 - 1 : 1;
  TC xn[nit<KB>()];
  prefetch_box<D, KB, TS, TC>(xn, xv + long(s0) * g.npts, n, ox, oy, oz);
  TC kr[FIX ? 1 : nit<KB>()][FIX ? 1 : RM];
  if constexpr (FIX) stage_fixed<D, KB, TC>(sk, L, g.nnodes, n, ox, oy, oz);
  else load_kraw<D, KB, TC, RM>(kr, (const TC*)L.kap, g.nnodes, L.R, n, ox, oy, oz);
  for (int s = s0; s < s1; ++s) {
    const TC gamma = FIX ? slab_scale<TC>(L, s) : TC(1);
    if constexpr (!FIX) write_kappa<KB, TC, RM>(sk, kr, level_op<TC>(L, s));
    write_box<KB, TC>(sx, xn);
    const TC sigma = L.sig ? ((const TC*)L.sig)[s] : TC(0);
    if (s + 1 < s1) prefetch_box<D, KB, TS, TC>(xn, xv + long(s + 1) * g.npts, n, ox, oy, oz);
    __syncthreads();
    TS* ys = yv + long(s) * g.npts;
    STP_BOX_FOR(TB, it) {
      const int jx = jx0 + it.x, jy = jy0 + it.y, jz = jz0 + it.z;
      if (!interior<D>(jx, jy, jz, n)) continue;
      const int kq = KB::idx(it.x + 1, D >= 2 ? it.y + 1 : 0, D >= 3 ? it.z + 1 : 0);
      const TC kc = sk[kq];
      TC dg = FIX ? TC(0) : sigma, off = 0;
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) {
        const TC w = kc + sk[kq + nb_off<KB>(k)];
        dg += w;
        off += w * sx[kq + nb_off<KB>(k)];
      }
      const TC y = FIX ? sigma * sx[kq] + gamma * (dg * sx[kq] - off) : dg * sx[kq] - off;
      const int vo = vec_off<D>(jx, jy, jz, n);
      st<TS, TC>(ys, vo, J.addout < 0 ? ld<TC>(ys, vo) - y : y);
      // between two cycles: the output so far takes the operand (o += x, or the
      // float64 p += x of the A-tilde cycles)
      if (acc) st<TS, TC>(acc + long(s) * g.npts, vo, ld<TC>(acc + long(s) * g.npts, vo) + sx[kq]);
      if (J.acc64) J.acc64[long(s) * g.npts + vo] += double(sx[kq]);
    }
    __syncthreads();
  }
}

template <int D, typename TS, typename TC, int RM, int V>
__global__ void __launch_bounds__(MidTile<D>::threads) k_apply_tile(const TileJob* __restrict__ jobs, int njobs) {
  int tile, s0, s1;
  const TileJob J = job_tile_run(jobs, njobs, 1 << 30, tile, s0, s1);
  if (J.state && done_flag(J.state)) return;
  if (job_fixed(V, J.op.cmode)) apply_tile_body<D, TS, TC, RM, true>(J, tile, s0, s1, (const TS*)J.b, (TS*)J.out);
  else apply_tile_body<D, TS, TC, RM, false>(J, tile, s0, s1, (const TS*)J.b, (TS*)J.out);
}

// ---------------------------------------------------------------------------
// time-global residuals (float64), tile versions marching forward in time
//   WHICH = 0 (a1):  r = (u_s - u_{s-1}) - tau_s A_s p_s - f_s
//   WHICH = 1 (a3):  e = f_s - (u_s - u_{s-1}) - tau_s A_s u_s,
//                    r = e - ((u+p)_s - (u+p)_{s+1}),  block partial of e^2
// f_s = tau_s F_s (+ u0 on the first slab).  The tile values of u_s are kept
// in registers and serve as u_{s-1} of the next slab.
// ---------------------------------------------------------------------------
template <int D, typename TS, int WHICH, int RM, bool FIX>
__device__ __forceinline__ void resid_tile_body(const ResidJob& J, int tile, int s0, int s1,
                                                const double* __restrict__ u, const double* __restrict__ p,
                                                const double* __restrict__ F, const double* __restrict__ u0,
                                                TS* __restrict__ r, double* __restrict__ partial) {
  using T = ResidTile<D>;
  using KB = Box<D, T::X + 2, T::Y + 2, T::Z + 2, T::threads>;
  using TB = Box<D, T::X, T::Y, T::Z, T::threads>;
  constexpr int NT = nit<TB>();
  __shared__ double sk[KB::size];
  __shared__ double sx[KB::size];
  const TimeOp t = J.t;
  s1 = min(s1, t.N);
  const Geom g = J.g;
  double e2 = 0.0;
  if (s0 < s1) {
    const int n = g.n;
    int tx, ty, tz;
    tile_origin<D, T>(n, tile, tx, ty, tz);
    const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
    const int ox = jx0 - 1, oy = D >= 2 ? jy0 - 1 : 1, oz = D >= 3 ? jz0 - 1 : 1;
    const double* X = WHICH == 0 ? p : u;   // operand of the stencil
    // per-thread tile offsets (-1: not an interior node of this tile)
    int vo[NT];
    {
      BoxIter<TB> it;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const int jx = jx0 + it.x, jy = jy0 + it.y, jz = jz0 + it.z;
        vo[k] = (it.ok() && interior<D>(jx, jy, jz, n)) ? vec_off<D>(jx, jy, jz, n) : -1;
        it.next();
      }
    }
    auto load_pts = [&](double (&v)[NT], const double* base) {
#pragma unroll
      for (int k = 0; k < NT; ++k) v[k] = vo[k] >= 0 ? base[vo[k]] : 0.0;
    };
    double kr[FIX ? 1 : nit<KB>()][FIX ? 1 : RM];
    if constexpr (FIX) {
      // rank 1: the field is staged once and scaled per slab by tau a_0[s]
      LevelOp L1{};
      L1.kap = t.kap;
      L1.c = t.cA;
      L1.R = 1;
      L1.cmode = CM_SCALE;
      stage_fixed<D, KB, double>(sk, L1, g.nnodes, n, ox, oy, oz);
    } else {
      load_kraw<D, KB, double, RM>(kr, t.kap, g.nnodes, t.R, n, ox, oy, oz);
    }
    double xn[nit<KB>()];
    prefetch_box<D, KB, double, double>(xn, X + long(s0) * g.npts, n, ox, oy, oz);
    // pointwise values of the current and the next slab
    double um[NT], uc[NT], un[NT], pc[NT], pn[NT], Fc[NT], Fn[NT];
    if (s0 > 0) load_pts(um, u + long(s0 - 1) * g.npts);
    else {
#pragma unroll
      for (int k = 0; k < NT; ++k) um[k] = 0.0;
    }
    load_pts(uc, u + long(s0) * g.npts);
    load_pts(Fc, F + long(s0) * g.npts);
    if (WHICH == 1) load_pts(pc, p + long(s0) * g.npts);
    for (int s = s0; s < s1; ++s) {
      const long o = long(s) * g.npts;
      const double tau = J.taus[s];
      const double gamma = FIX ? t.cA[s * kMaxRank] : 1.0;
      if constexpr (!FIX) write_kappa<KB, double, RM>(sk, kr, load_op<double>(nullptr, t.cA, s, t.R));
      write_box<KB, double>(sx, xn);
      const bool more = s + 1 < t.N;          // slab s+1 exists
      if (more) {
        const long o1 = o + g.npts;
        if (s + 1 < s1) prefetch_box<D, KB, double, double>(xn, X + o1, n, ox, oy, oz);
        load_pts(un, u + o1);
        if (s + 1 < s1) load_pts(Fn, F + o1);
        if (WHICH == 1) load_pts(pn, p + o1);
      }
      __syncthreads();
      TS* rs = r + o;
      BoxIter<TB> it;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (vo[k] >= 0) {
          const int kq = KB::idx(it.x + 1, D >= 2 ? it.y + 1 : 0, D >= 3 ? it.z + 1 : 0);
          const double kc = sk[kq];
          double dg = 0, off = 0;
#pragma unroll
          for (int q = 0; q < 2 * D; ++q) {
            const double w = kc + sk[kq + nb_off<KB>(q)];
            dg += w;
            off += w * sx[kq + nb_off<KB>(q)];
          }
          const double Ax = FIX ? gamma * (dg * sx[kq] - off) : dg * sx[kq] - off;
          double f = tau * Fc[k];
          if (s == 0) f += u0[vo[k]];
          if (WHICH == 0) {
            st<TS, double>(rs, vo[k], (uc[k] - um[k]) - Ax - f);
          } else {
            const double e = f - (uc[k] - um[k]) - Ax;
            const double wn = more ? un[k] + pn[k] : 0.0;
            st<TS, double>(rs, vo[k], e - ((uc[k] + pc[k]) - wn));
            e2 += e * e;
          }
        }
        it.next();
      }
      __syncthreads();
      // march: the current slab becomes the previous one
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        um[k] = uc[k];
        uc[k] = un[k];
        Fc[k] = Fn[k];
        if (WHICH == 1) pc[k] = pn[k];
      }
    }
  }
  if (WHICH == 1) {
    const double bs = block_sum<ResidTile<D>::threads>(e2);
    if (threadIdx.x == 0) partial[block_id() - J.block0] = bs;
  }
}

template <int D, typename TS, int WHICH, int RM, int V>
__global__ void __launch_bounds__(ResidTile<D>::threads) k_resid_tile(const ResidJob* __restrict__ jobs, int njobs) {
  int tile, s0, s1;
  const ResidJob J = job_tile_run(jobs, njobs, 1 << 30, tile, s0, s1);
  if (J.state && done_flag(J.state)) return;
  // the residual's operator is the A family: a fixed field when the rank is 1
  if (job_fixed(V, J.t.R == 1 ? CM_SCALE : CM_SLAB))
    resid_tile_body<D, TS, WHICH, RM, true>(J, tile, s0, s1, J.u, J.p, J.F, J.u0, (TS*)J.r, J.partial);
  else
    resid_tile_body<D, TS, WHICH, RM, false>(J, tile, s0, s1, J.u, J.p, J.F, J.u0, (TS*)J.r, J.partial);
}

// ---------------------------------------------------------------------------
// ||r_p||^2 and ||r_u||^2 of a pair (u, p), eq. (3.1), on the up-sweep tiles:
//   r_p = K u - A p - f,  r_u = f - K^T p - (K + K^T + A) u.
// Both stencil operands (p and u) are staged per slab with their halo; a
// block walks its slab run with u_{s-1}, u_{s+1} and p_{s+1} in registers and
// writes partial[b] (r_p) and partial[count + b] (r_u) for its job-local
// block b.  One pass over u, p and F after a solve.
// ---------------------------------------------------------------------------
template <int D, int RM, bool FIX>
__device__ __forceinline__ void pair_norms_body(const ResidJob& J, int tile, int s0, int s1, long count) {
  using T = UpTile<D>;
  using KB = Box<D, T::X + 2, T::Y + 2, T::Z + 2>;
  using TB = Box<D, T::X, T::Y, T::Z>;
  constexpr int NT = nit<TB>();
  __shared__ double sk[KB::size];
  __shared__ double sp[KB::size];
  __shared__ double su[KB::size];
  const TimeOp t = J.t;
  s1 = min(s1, t.N);
  const Geom g = J.g;
  const double* u = J.u;
  const double* p = J.p;
  double vp = 0.0, vu = 0.0;
  if (s0 < s1) {
    const int n = g.n;
    int tx, ty, tz;
    tile_origin<D, T>(n, tile, tx, ty, tz);
    const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
    const int ox = jx0 - 1, oy = D >= 2 ? jy0 - 1 : 1, oz = D >= 3 ? jz0 - 1 : 1;
    int vo[NT];
    {
      BoxIter<TB> it;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const int jx = jx0 + it.x, jy = jy0 + it.y, jz = jz0 + it.z;
        vo[k] = (it.ok() && interior<D>(jx, jy, jz, n)) ? vec_off<D>(jx, jy, jz, n) : -1;
        it.next();
      }
    }
    auto load_pts = [&](double(&v)[NT], const double* base) {
#pragma unroll
      for (int k = 0; k < NT; ++k) v[k] = vo[k] >= 0 ? base[vo[k]] : 0.0;
    };
    double kr[FIX ? 1 : nit<KB>()][FIX ? 1 : RM];
    if constexpr (FIX) {
      LevelOp L1{};
      L1.kap = t.kap;
      L1.c = t.cA;
      L1.R = 1;
      L1.cmode = CM_SCALE;
      stage_fixed<D, KB, double>(sk, L1, g.nnodes, n, ox, oy, oz);
    } else {
      load_kraw<D, KB, double, RM>(kr, t.kap, g.nnodes, t.R, n, ox, oy, oz);
    }
    double pn_box[nit<KB>()], un_box[nit<KB>()];
    prefetch_box<D, KB, double, double>(pn_box, p + long(s0) * g.npts, n, ox, oy, oz);
    prefetch_box<D, KB, double, double>(un_box, u + long(s0) * g.npts, n, ox, oy, oz);
    double um[NT], uk[NT], Fc[NT], Fn[NT], un[NT], pn[NT];
    if (s0 > 0) load_pts(um, u + long(s0 - 1) * g.npts);
    else {
#pragma unroll
      for (int k = 0; k < NT; ++k) um[k] = 0.0;
    }
    load_pts(Fc, J.F + long(s0) * g.npts);
    for (int s = s0; s < s1; ++s) {
      const long o = long(s) * g.npts;
      const double tau = J.taus[s];
      const double gamma = FIX ? t.cA[s * kMaxRank] : 1.0;
      if constexpr (!FIX) write_kappa<KB, double, RM>(sk, kr, load_op<double>(nullptr, t.cA, s, t.R));
      write_box<KB, double>(sp, pn_box);
      write_box<KB, double>(su, un_box);
      const bool more = s + 1 < t.N;
      if (more) {
        const long o1 = o + g.npts;
        if (s + 1 < s1) {
          prefetch_box<D, KB, double, double>(pn_box, p + o1, n, ox, oy, oz);
          prefetch_box<D, KB, double, double>(un_box, u + o1, n, ox, oy, oz);
          load_pts(Fn, J.F + o1);
        }
        load_pts(un, u + o1);
        load_pts(pn, p + o1);
      }
      __syncthreads();
      BoxIter<TB> it;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (vo[k] >= 0) {
          const int kq = KB::idx(it.x + 1, D >= 2 ? it.y + 1 : 0, D >= 3 ? it.z + 1 : 0);
          const double kc = sk[kq];
          double dg = 0, offp = 0, offu = 0;
#pragma unroll
          for (int q = 0; q < 2 * D; ++q) {
            const double w = kc + sk[kq + nb_off<KB>(q)];
            dg += w;
            offp += w * sp[kq + nb_off<KB>(q)];
            offu += w * su[kq + nb_off<KB>(q)];
          }
          const double pc = sp[kq], uc = su[kq];
          uk[k] = uc;
          const double Ap = FIX ? gamma * (dg * pc - offp) : dg * pc - offp;
          const double Au = FIX ? gamma * (dg * uc - offu) : dg * uc - offu;
          double f = tau * Fc[k];
          if (s == 0) f += J.u0[vo[k]];
          const double up = more ? un[k] : 0.0, pp = more ? pn[k] : 0.0;
          const double rp = (uc - um[k]) - Ap - f;
          const double ru = f - (pc - pp) - (2.0 * uc - um[k] - up) - Au;
          vp += rp * rp;
          vu += ru * ru;
        }
        it.next();
      }
      __syncthreads();   // the next slab rewrites the staged boxes
      // march: u_s (the staged centre) becomes u_{s-1}
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        um[k] = vo[k] >= 0 ? uk[k] : 0.0;
        Fc[k] = Fn[k];
      }
    }
  }
  const long b = block_id() - J.block0;
  const double bp = block_sum(vp);
  if (threadIdx.x == 0) J.partial[b] = bp;
  __syncthreads();   // block_sum's LDS slots are reused
  const double bu = block_sum(vu);
  if (threadIdx.x == 0) J.partial[count + b] = bu;
}

// one job per problem; count: the job's blocks (the offset of the r_u row)
template <int D, int RM, int V>
__global__ void __launch_bounds__(kBlock) k_pair_norms(const ResidJob* __restrict__ jobs, int njobs) {
  int tile, s0, s1;
  const ResidJob J = job_tile_run(jobs, njobs, 1 << 30, tile, s0, s1);
  const long count = long(J.tiles) * ((J.t.N + J.sb - 1) / J.sb);
  if (job_fixed(V, J.t.R == 1 ? CM_SCALE : CM_SLAB)) pair_norms_body<D, RM, true>(J, tile, s0, s1, count);
  else pair_norms_body<D, RM, false>(J, tile, s0, s1, count);
}

}  // namespace stp

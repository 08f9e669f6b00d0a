// LDS-tiled stencil kernels: the fused multigrid level kernels and the
// time-global residual kernels.
//
// Every block owns one spatial tile of one slab.  It stages into LDS the
// slab-combined coefficient kappa_s = sum_r c_{s,r} k_r (k_r = kappa_r / 2h^2,
// nodal, incl. boundary) over the tile plus the halo its stencils need, so a
// face weight is kappa_s[i] + kappa_s[nb] and the diagonal is
// sigma_s + sum over the 2d faces.
//
// Node coordinates are 1-based with 0 and n+1 on the boundary; interior
// vector entry of node j sits at offset j-1 per axis.
#pragma once
#include "stp_kernels.h"

namespace stp {

template <int D, int EX, int EY, int EZ>
struct Box {
  static constexpr int X = EX;
  static constexpr int Y = (D >= 2 ? EY : 1);
  static constexpr int Z = (D >= 3 ? EZ : 1);
  static constexpr int size = X * Y * Z;
  __device__ static __forceinline__ void coords(int q, int& x, int& y, int& z) {
    x = q % X;
    y = (q / X) % Y;
    z = q / (X * Y);
  }
  __device__ static __forceinline__ int idx(int x, int y, int z) { return (z * Y + y) * X + x; }
};

// offsets of the 2d neighbours inside a box (x-, x+, y-, y+, z-, z+)
template <int D, typename B>
__device__ __forceinline__ int nb_off(int k) {
  switch (k) {
    case 0: return -1;
    case 1: return 1;
    case 2: return -B::X;
    case 3: return B::X;
    case 4: return -B::X * B::Y;
    default: return B::X * B::Y;
  }
}

template <int D>
__device__ __forceinline__ long node_index(int jx, int jy, int jz, long nn) {
  if (D == 1) return jx;
  if (D == 2) return long(jy) * nn + jx;
  return (long(jz) * nn + jy) * nn + jx;
}

template <int D>
__device__ __forceinline__ long vec_index(int jx, int jy, int jz, long n) {
  // interior node (1-based) -> vector offset within a slab
  if (D == 1) return jx - 1;
  if (D == 2) return long(jy - 1) * n + (jx - 1);
  return (long(jz - 1) * n + (jy - 1)) * n + (jx - 1);
}

template <int D>
__device__ __forceinline__ bool in_nodes(int jx, int jy, int jz, int n) {
  bool ok = jx >= 0 && jx <= n + 1;
  if (D >= 2) ok = ok && jy >= 0 && jy <= n + 1;
  if (D >= 3) ok = ok && jz >= 0 && jz <= n + 1;
  return ok;
}

template <int D>
__device__ __forceinline__ bool interior(int jx, int jy, int jz, int n) {
  bool ok = jx >= 1 && jx <= n;
  if (D >= 2) ok = ok && jy >= 1 && jy <= n;
  if (D >= 3) ok = ok && jz >= 1 && jz <= n;
  return ok;
}

// Stage kappa_s over box KB whose origin is node (ox, oy, oz).
template <int D, typename KB, typename TC>
__device__ __forceinline__ void stage_kappa(TC* sk, const TC* __restrict__ kap, long nnodes, int n, int ox, int oy,
                                            int oz, const SlabOp<TC>& op, int R) {
  const long nn = n + 2;
  for (int q = threadIdx.x; q < KB::size; q += kBlock) {
    int x, y, z;
    KB::coords(q, x, y, z);
    const int jx = ox + x, jy = oy + y, jz = oz + z;
    TC v = 0;
    if (in_nodes<D>(jx, jy, jz, n)) v = kmix(kap, nnodes, node_index<D>(jx, jy, jz, nn), op, R);
    sk[q] = v;
  }
}

// diagonal and off-diagonal sum at box position q of box XB, whose kappa box KB
// is shifted by one node in every active axis.
template <int D, typename XB, typename KB, typename TC>
__device__ __forceinline__ TC diag_box(const TC* sk, int x, int y, int z, TC sigma) {
  const int kq = KB::idx(x + 1, D >= 2 ? y + 1 : 0, D >= 3 ? z + 1 : 0);
  const TC kc = sk[kq];
  TC d = sigma + TC(2 * D) * kc;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) d += sk[kq + nb_off<D, KB>(k)];
  return d;
}

template <int D, typename XB, typename KB, typename TC>
__device__ __forceinline__ TC offsum_box(const TC* sk, const TC* sx, int x, int y, int z) {
  const int kq = KB::idx(x + 1, D >= 2 ? y + 1 : 0, D >= 3 ? z + 1 : 0);
  const int xq = XB::idx(x, y, z);
  const TC kc = sk[kq];
  TC o = 0;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) o += (kc + sk[kq + nb_off<D, KB>(k)]) * sx[xq + nb_off<D, XB>(k)];
  return o;
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

template <int D, typename T>
__host__ __device__ inline long tiles_for(int n) {
  long t = (n + T::X - 1) / T::X;
  if (D >= 2) t *= (n + T::Y - 1) / T::Y;
  if (D >= 3) t *= (n + T::Z - 1) / T::Z;
  return t;
}

template <int D, typename T>
__device__ __forceinline__ void tile_origin(int n, int& tx, int& ty, int& tz) {
  const int ntx = (n + T::X - 1) / T::X;
  const int nty = D >= 2 ? (n + T::Y - 1) / T::Y : 1;
  int t = blockIdx.x;
  tx = t % ntx;
  t /= ntx;
  ty = D >= 2 ? t % nty : 0;
  tz = D >= 3 ? t / nty : 0;
}

// ---------------------------------------------------------------------------
// multigrid: pre-smooth from zero, residual and full-weighting restriction
//   x1 = omega D^{-1} b,  r = b - L x1,  bc = R r
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_mg_down(Geom gf, Geom gc, LevelOp L, TC omega, const TS* __restrict__ b,
                                                    TS* __restrict__ bc, const int* __restrict__ state) {
  if (state && done_flag(state)) return;
  using T = DownTile<D>;
  using KB = Box<D, 2 * T::X + 5, 2 * T::Y + 5, 2 * T::Z + 5>;
  using XB = Box<D, 2 * T::X + 3, 2 * T::Y + 3, 2 * T::Z + 3>;
  using RB = Box<D, 2 * T::X + 1, 2 * T::Y + 1, 2 * T::Z + 1>;
  using CB = Box<D, T::X, T::Y, T::Z>;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[XB::size];
  __shared__ TC sr[RB::size];
  const int s = slab_index();
  if (s >= L.S) return;
  const int nf = gf.n, nc = gc.n;
  int tx, ty, tz;
  tile_origin<D, T>(nc, tx, ty, tz);
  // first coarse node of the tile (1-based); fine node of coarse I is 2I
  const int Ix = tx * T::X + 1, Iy = D >= 2 ? ty * T::Y + 1 : 1, Iz = D >= 3 ? tz * T::Z + 1 : 1;
  const int rx = 2 * Ix - 1, ry = D >= 2 ? 2 * Iy - 1 : 1, rz = D >= 3 ? 2 * Iz - 1 : 1;   // r-box origin
  const int xx = rx - 1, xy = D >= 2 ? ry - 1 : 1, xz = D >= 3 ? rz - 1 : 1;                // x1-box origin
  const int kx = xx - 1, ky = D >= 2 ? xy - 1 : 1, kz = D >= 3 ? xz - 1 : 1;                // kappa-box origin
  const SlabOp<TC> op = level_op<TC>(L, s);
  stage_kappa<D, KB, TC>(sk, (const TC*)L.kap, gf.nnodes, nf, kx, ky, kz, op, L.R);
  __syncthreads();
  const TS* bs = b + long(s) * gf.npts;
  for (int q = threadIdx.x; q < XB::size; q += kBlock) {
    int x, y, z;
    XB::coords(q, x, y, z);
    const int jx = xx + x, jy = xy + y, jz = xz + z;
    TC v = 0;
    if (interior<D>(jx, jy, jz, nf)) {
      const TC dg = diag_box<D, XB, KB, TC>(sk, x, y, z, op.sigma);
      v = omega * ld<TC>(bs, vec_index<D>(jx, jy, jz, nf)) / dg;
    }
    sx[q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < RB::size; q += kBlock) {
    int x, y, z;
    RB::coords(q, x, y, z);
    const int jx = rx + x, jy = ry + y, jz = rz + z;
    TC v = 0;
    if (interior<D>(jx, jy, jz, nf)) {
      // box position of this node inside the x1 box is (x+1, y+1, z+1)
      const int ax = x + 1, ay = D >= 2 ? y + 1 : 0, az = D >= 3 ? z + 1 : 0;
      const TC dg = diag_box<D, XB, KB, TC>(sk, ax, ay, az, op.sigma);
      const TC off = offsum_box<D, XB, KB, TC>(sk, sx, ax, ay, az);
      v = ld<TC>(bs, vec_index<D>(jx, jy, jz, nf)) - (dg * sx[XB::idx(ax, ay, az)] - off);
    }
    sr[q] = v;
  }
  __syncthreads();
  TS* bcs = bc + long(s) * gc.npts;
  for (int q = threadIdx.x; q < CB::size; q += kBlock) {
    int x, y, z;
    CB::coords(q, x, y, z);
    const int Jx = Ix + x, Jy = Iy + y, Jz = Iz + z;
    if (!interior<D>(Jx, Jy, Jz, nc)) continue;
    // fine node 2J sits at r-box position 2x+1 per axis
    const int cx = 2 * x + 1, cy = D >= 2 ? 2 * y + 1 : 0, cz = D >= 3 ? 2 * z + 1 : 0;
    TC acc = 0;
#pragma unroll
    for (int dz = (D >= 3 ? -1 : 0); dz <= (D >= 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          TC w = (dx == 0 ? TC(0.5) : TC(0.25));
          if (D >= 2) w *= (dy == 0 ? TC(0.5) : TC(0.25));
          if (D >= 3) w *= (dz == 0 ? TC(0.5) : TC(0.25));
          acc += w * sr[RB::idx(cx + dx, cy + dy, cz + dz)];
        }
    st<TS, TC>(bcs, vec_index<D>(Jx, Jy, Jz, nc), acc);
  }
}

// ---------------------------------------------------------------------------
// multigrid: coarse correction and post-smoothing
//   x2 = omega D^{-1} b + P e,   x = x2 + omega D^{-1} (b - L x2)
// epilogue: store x (TS) or add it into a float64 vector
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC, int EPI>
__global__ void __launch_bounds__(kBlock) k_mg_up(Geom gf, Geom gc, LevelOp L, TC omega, const TS* __restrict__ b,
                                                  const TS* __restrict__ e, TS* __restrict__ out,
                                                  double* __restrict__ acc64, const int* __restrict__ state) {
  if (state && done_flag(state)) return;
  using T = UpTile<D>;
  using KB = Box<D, T::X + 4, T::Y + 4, T::Z + 4>;
  using XB = Box<D, T::X + 2, T::Y + 2, T::Z + 2>;
  using EB = Box<D, T::X / 2 + 2, T::Y / 2 + 2, T::Z / 2 + 2>;
  using TB = Box<D, T::X, T::Y, T::Z>;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[XB::size];
  __shared__ TC sb[XB::size];
  __shared__ TC se[EB::size];
  const int s = slab_index();
  if (s >= L.S) return;
  const int nf = gf.n, nc = gc.n;
  int tx, ty, tz;
  tile_origin<D, T>(nf, tx, ty, tz);
  const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
  const int xx = jx0 - 1, xy = D >= 2 ? jy0 - 1 : 1, xz = D >= 3 ? jz0 - 1 : 1;   // x2-box origin
  const int kx = xx - 1, ky = D >= 2 ? xy - 1 : 1, kz = D >= 3 ? xz - 1 : 1;      // kappa-box origin
  const int ex = xx / 2, ey = D >= 2 ? xy / 2 : 1, ez = D >= 3 ? xz / 2 : 1;      // first coarse node
  const SlabOp<TC> op = level_op<TC>(L, s);
  stage_kappa<D, KB, TC>(sk, (const TC*)L.kap, gf.nnodes, nf, kx, ky, kz, op, L.R);
  const TS* es = e + long(s) * gc.npts;
  for (int q = threadIdx.x; q < EB::size; q += kBlock) {
    int x, y, z;
    EB::coords(q, x, y, z);
    const int Jx = ex + x, Jy = ey + y, Jz = ez + z;
    se[q] = interior<D>(Jx, Jy, Jz, nc) ? ld<TC>(es, vec_index<D>(Jx, Jy, Jz, nc)) : TC(0);
  }
  __syncthreads();
  const TS* bs = b + long(s) * gf.npts;
  for (int q = threadIdx.x; q < XB::size; q += kBlock) {
    int x, y, z;
    XB::coords(q, x, y, z);
    const int jx = xx + x, jy = xy + y, jz = xz + z;
    TC v = 0, bv = 0;
    if (interior<D>(jx, jy, jz, nf)) {
      bv = ld<TC>(bs, vec_index<D>(jx, jy, jz, nf));
      const TC dg = diag_box<D, XB, KB, TC>(sk, x, y, z, op.sigma);
      // multilinear interpolation from coarse nodes floor(j/2), ceil(j/2)
      const int lx = (jx >> 1) - ex, ly = D >= 2 ? (jy >> 1) - ey : 0, lz = D >= 3 ? (jz >> 1) - ez : 0;
      const int ox = jx & 1, oy = D >= 2 ? (jy & 1) : 0, oz = D >= 3 ? (jz & 1) : 0;
      TC pe = 0;
#pragma unroll
      for (int az = 0; az <= (D >= 3 ? 1 : 0); ++az)
#pragma unroll
        for (int ay = 0; ay <= (D >= 2 ? 1 : 0); ++ay)
#pragma unroll
          for (int ax = 0; ax <= 1; ++ax) {
            if ((ax && !ox) || (ay && !oy) || (az && !oz)) continue;
            TC w = ox ? TC(0.5) : TC(1);
            if (D >= 2) w *= oy ? TC(0.5) : TC(1);
            if (D >= 3) w *= oz ? TC(0.5) : TC(1);
            pe += w * se[EB::idx(lx + ax, ly + ay, lz + az)];
          }
      v = omega * bv / dg + pe;
    }
    sx[q] = v;
    sb[q] = bv;
  }
  __syncthreads();
  const long o = long(s) * gf.npts;
  for (int q = threadIdx.x; q < TB::size; q += kBlock) {
    int x, y, z;
    TB::coords(q, x, y, z);
    const int jx = jx0 + x, jy = jy0 + y, jz = jz0 + z;
    if (!interior<D>(jx, jy, jz, nf)) continue;
    const int ax = x + 1, ay = D >= 2 ? y + 1 : 0, az = D >= 3 ? z + 1 : 0;
    const int xq = XB::idx(ax, ay, az);
    const TC dg = diag_box<D, XB, KB, TC>(sk, ax, ay, az, op.sigma);
    const TC off = offsum_box<D, XB, KB, TC>(sk, sx, ax, ay, az);
    const TC x2 = sx[xq];
    const TC v = x2 + omega * (sb[xq] - (dg * x2 - off)) / dg;
    const long vi = o + vec_index<D>(jx, jy, jz, nf);
    if (EPI == EPI_STORE) st<TS, TC>(out, vi, v);
    else acc64[vi] += double(v);
  }
}

// ---------------------------------------------------------------------------
// y = L x (tile version; the middle reference operator of the H-blocks)
// ---------------------------------------------------------------------------
template <int D, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_apply_tile(Geom g, LevelOp L, const TS* __restrict__ xv,
                                                       TS* __restrict__ yv, const int* __restrict__ state) {
  if (state && done_flag(state)) return;
  using T = UpTile<D>;
  using KB = Box<D, T::X + 2, T::Y + 2, T::Z + 2>;
  using XB = KB;
  using TB = Box<D, T::X, T::Y, T::Z>;
  __shared__ TC sk[KB::size];
  __shared__ TC sx[XB::size];
  const int s = slab_index();
  if (s >= L.S) return;
  const int n = g.n;
  int tx, ty, tz;
  tile_origin<D, T>(n, tx, ty, tz);
  const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
  const int ox = jx0 - 1, oy = D >= 2 ? jy0 - 1 : 1, oz = D >= 3 ? jz0 - 1 : 1;
  const SlabOp<TC> op = level_op<TC>(L, s);
  const TS* xs = xv + long(s) * g.npts;
  const long nn = n + 2;
  for (int q = threadIdx.x; q < KB::size; q += kBlock) {
    int x, y, z;
    KB::coords(q, x, y, z);
    const int jx = ox + x, jy = oy + y, jz = oz + z;
    TC kv = 0, v = 0;
    if (in_nodes<D>(jx, jy, jz, n)) {
      kv = kmix((const TC*)L.kap, g.nnodes, node_index<D>(jx, jy, jz, nn), op, L.R);
      if (interior<D>(jx, jy, jz, n)) v = ld<TC>(xs, vec_index<D>(jx, jy, jz, n));
    }
    sk[q] = kv;
    sx[q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < TB::size; q += kBlock) {
    int x, y, z;
    TB::coords(q, x, y, z);
    const int jx = jx0 + x, jy = jy0 + y, jz = jz0 + z;
    if (!interior<D>(jx, jy, jz, n)) continue;
    const int ax = x + 1, ay = D >= 2 ? y + 1 : 0, az = D >= 3 ? z + 1 : 0;
    const int kq = KB::idx(ax, ay, az);
    const TC kc = sk[kq];
    TC dg = op.sigma, off = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      const TC w = kc + sk[kq + nb_off<D, KB>(k)];
      dg += w;
      off += w * sx[kq + nb_off<D, KB>(k)];
    }
    st<TS, TC>(yv, long(s) * g.npts + vec_index<D>(jx, jy, jz, n), dg * sx[kq] - off);
  }
}

// ---------------------------------------------------------------------------
// time-global residuals (float64), tile versions
//   WHICH = 0 (a1):  r = (u_s - u_{s-1}) - tau A_s p_s - f_s
//   WHICH = 1 (a3):  e = f_s - (u_s - u_{s-1}) - tau A_s u_s,
//                    r = e - ((u+p)_s - (u+p)_{s+1}),  block partial of e^2
// ---------------------------------------------------------------------------
template <int D, typename TS, int WHICH>
__global__ void __launch_bounds__(kBlock) k_resid_tile(Geom g, TimeOp t, double tau, const double* __restrict__ u,
                                                       const double* __restrict__ p, const double* __restrict__ F,
                                                       const double* __restrict__ u0, TS* __restrict__ r,
                                                       double* __restrict__ partial, const int* __restrict__ state) {
  if (state && done_flag(state)) return;
  using T = UpTile<D>;
  using KB = Box<D, T::X + 2, T::Y + 2, T::Z + 2>;
  using TB = Box<D, T::X, T::Y, T::Z>;
  __shared__ double sk[KB::size];
  __shared__ double sx[KB::size];
  const int s = slab_index();
  double e2 = 0.0;
  if (s < t.N) {
    const int n = g.n;
    int tx, ty, tz;
    tile_origin<D, T>(n, tx, ty, tz);
    const int jx0 = tx * T::X + 1, jy0 = D >= 2 ? ty * T::Y + 1 : 1, jz0 = D >= 3 ? tz * T::Z + 1 : 1;
    const int ox = jx0 - 1, oy = D >= 2 ? jy0 - 1 : 1, oz = D >= 3 ? jz0 - 1 : 1;
    const SlabOp<double> op = load_op<double>(nullptr, t.cA, s, t.R);
    const long o = long(s) * g.npts;
    const double* xs = (WHICH == 0 ? p : u) + o;   // operand of the stencil
    const long nn = n + 2;
    for (int q = threadIdx.x; q < KB::size; q += kBlock) {
      int x, y, z;
      KB::coords(q, x, y, z);
      const int jx = ox + x, jy = oy + y, jz = oz + z;
      double kv = 0, v = 0;
      if (in_nodes<D>(jx, jy, jz, n)) {
        kv = kmix(t.kap, g.nnodes, node_index<D>(jx, jy, jz, nn), op, t.R);
        if (interior<D>(jx, jy, jz, n)) v = xs[vec_index<D>(jx, jy, jz, n)];
      }
      sk[q] = kv;
      sx[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < TB::size; q += kBlock) {
      int x, y, z;
      TB::coords(q, x, y, z);
      const int jx = jx0 + x, jy = jy0 + y, jz = jz0 + z;
      if (!interior<D>(jx, jy, jz, n)) continue;
      const int ax = x + 1, ay = D >= 2 ? y + 1 : 0, az = D >= 3 ? z + 1 : 0;
      const int kq = KB::idx(ax, ay, az);
      const double kc = sk[kq];
      double dg = 0, off = 0;
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) {
        const double w = kc + sk[kq + nb_off<D, KB>(k)];
        dg += w;
        off += w * sx[kq + nb_off<D, KB>(k)];
      }
      const double Ax = dg * sx[kq] - off;
      const long vi = vec_index<D>(jx, jy, jz, n);
      const double uc = WHICH == 0 ? u[o + vi] : sx[kq];
      const double um = s > 0 ? u[o - g.npts + vi] : 0.0;
      double f = tau * F[o + vi];
      if (s == 0) f += u0[vi];
      if (WHICH == 0) {
        st<TS, double>(r, o + vi, (uc - um) - Ax - f);
      } else {
        const double e = f - (uc - um) - Ax;
        const double w = uc + p[o + vi];
        const double wn = s + 1 < t.N ? u[o + g.npts + vi] + p[o + g.npts + vi] : 0.0;
        st<TS, double>(r, o + vi, e - (w - wn));
        e2 += e * e;
      }
    }
  }
  if (WHICH == 1) {
    const double bs = block_sum(e2);
    if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
  }
}

}  // namespace stp

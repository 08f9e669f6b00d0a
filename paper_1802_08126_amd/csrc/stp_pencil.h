// 3-D multigrid level sweeps as register pencils (fixed-field levels): the
// down-sweep (pre-smoothing from zero, residual, full-weighting restriction)
// and the up-sweep (prolongation, coarse correction, post-smoothing).
//
// The LDS-tiled down-sweep stages a 3-D box of x1 = omega D^{-1} b per block
// and recomputes its halo 2.25 times over; it is bound by instruction issue,
// not by HBM.  These kernels keep every value in registers instead:
//
//   - a wave owns a pencil: up to 30 coarse nodes along x (its 64 lanes are
//     the fine nodes 2 I0 - 2 .. 2 I0 + 61), TY coarse rows along y (2 TY + 3
//     fine rows per lane, one register each) and TZ coarse planes along z,
//     which it marches plane by plane with a three-plane register ring;
//   - x-neighbours come from the adjacent lanes through DPP wave shifts,
//     y-neighbours from the lane's other rows, z-neighbours from the ring, so
//     the kernel has no LDS traffic and no barriers;
//   - the four waves of a block are four consecutive slabs of the same
//     pencil, so the slab-independent fields are read from HBM once and then
//     hit in L1/L2 for the other three;
//   - the per-level fields are precomputed: k (the fixed coefficient field at
//     the interior nodes) and d (its face sum 2d k_c + sum_nb k_nb, boundary
//     neighbours included), so the diagonal of slab s is sigma_s + gamma_s d;
//   - loads go through buffer descriptors: the row/plane offset is a scalar
//     operand and lanes outside the domain read zero through the range check.
//
// Arithmetic per fine node is that of the tiled kernel (x1, the six-face
// residual in the same order); the full-weighting restriction is summed z
// first, then y, then x.
#pragma once
#include <type_traits>

#include "stp_tiles.h"

namespace stp {

constexpr int kPencilWaves = 4;     // waves (slabs) per block
constexpr int kPencilPasses = 1;    // slabs each wave marches in turn
constexpr int kPencilSlabs = kPencilWaves * kPencilPasses;   // slabs per block
constexpr int kPencilThreads = 64 * kPencilWaves;
// Block order: consecutive blocks take consecutive pencils of one slab group
// (true: the slab groups of one pencil), x-segments fastest, then y-tiles, so
// the pencils next to each other in x and y, which share halo lines and rows,
// run at the same time on one L2.  On 255^3 x 64 (float32, level 0) this order
// took the down-sweep from 2.70 ms (slab groups fastest) to 2.38 (y fastest)
// and 2.22 ms; two or more passes of slabs per wave were slower.
constexpr bool kPencilGroupFastest = false;
constexpr bool kPencilXFastest = true;
// planes of loads in flight ahead of the down-sweep's march: one took 2.11 ms
// against two planes' 2.22 (float32, four rows), the freed registers paying for
// taller pencils
constexpr int kPencilDepth = 1;
constexpr int kPencilCX = 30;       // coarse nodes per wave along x (2 * 30 + 3 lanes used)
constexpr int kPencilTZ = 16;       // coarse planes per wave
constexpr int kPencilMinNc = 24;    // coarser levels keep the tiled kernel (lanes would idle)

// coarse rows per pencil, set by measurement on 255^3 x 64: the down-sweep
// (PencilTY) gains from taller pencils (fewer halo rows per owned row) while its
// registers allow; the up-sweep storing a level (PencilUpTY, EPI_STORE) is
// fastest at four rows, the ones adding into the float64 iterate or into their
// output at two (the extra read-modify-write wants the occupancy of ~144 VGPRs)
template <typename TC> struct PencilTY;
template <> struct PencilTY<float> { static constexpr int v = 6; };
template <> struct PencilTY<double> { static constexpr int v = 4; };
template <typename TS, int EPI> struct PencilUpTY { static constexpr int v = EPI == EPI_STORE ? 4 : 2; };
template <int EPI> struct PencilUpTY<double, EPI> { static constexpr int v = 2; };
// bfloat16 storage: two rows for both up-sweeps (the storing one needs 302 VGPRs
// at four rows, one wave per SIMD, and took 9.5 ms against the tiles' 7.4; at two
// rows, 146 VGPRs, 3.0 ms)
template <int EPI> struct PencilUpTY<bf16, EPI> { static constexpr int v = 2; };
// rows of the up-sweep pencil for a run-time epilogue (host-side tile counts)
template <typename TS>
constexpr int pencil_up_ty(int epi) {
  return epi == EPI_STORE ? PencilUpTY<TS, EPI_STORE>::v
         : epi == EPI_ADD64 ? PencilUpTY<TS, EPI_ADD64>::v : PencilUpTY<TS, EPI_ADDTS>::v;
}

// pencils of a level with nc coarse nodes per axis
__host__ __device__ inline long pencil_tiles(int nc, int ty) {
  const long nxs = (nc + kPencilCX - 1) / kPencilCX;
  const long nyt = (nc + ty - 1) / ty;
  const long nzt = (nc + kPencilTZ - 1) / kPencilTZ;
  return nxs * nyt * nzt;
}

// wave_shr:1 / wave_shl:1 - lane i reads lane i - 1 / i + 1 (zero past the ends)
constexpr int kDppFromLower = 0x138;
constexpr int kDppFromUpper = 0x130;

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(u)), CTRL, 0xf, 0xf, true));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(u >> 32)), CTRL, 0xf, 0xf, true));
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

using rsrc_t = __amdgpu_buffer_rsrc_t;

// raw buffer of `bytes` bytes at p (bytes < 2^31); offsets at or past the end read 0
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), 0x00020000);
}

template <typename TC, typename T>
__device__ __forceinline__ TC bload(rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float, float>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}
template <>
__device__ __forceinline__ double bload<double, double>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
}
template <>
__device__ __forceinline__ float bload<float, bf16>(rsrc_t r, unsigned voff, unsigned soff) {
  return bf16_to_f(bf16{uint16_t(__builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), 0))});
}

// Per-level fields of a fixed-field family: kf = sum_r f_r k_r at the interior
// nodes and df = 2d kf_c + sum_nb kf_nb (boundary neighbours included), in the
// arithmetic order of the tiled kernels' staging.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_pencil_fields(Geom g, LevelOp L, TC* __restrict__ kf,
                                                          TC* __restrict__ df) {
  const int n = g.n;
  const TC* kap = (const TC*)L.kap;
  TC f[kMaxRank];
#pragma unroll
  for (int r = 0; r < kMaxRank; ++r) f[r] = r < L.R ? fixed_coef<TC>(L, r) : TC(0);
  auto node = [&](int jx, int jy, int jz) {
    const int o = node_off<3>(jx, jy, jz, n);
    TC v = f[0] * kap[o];
    for (int r = 1; r < L.R; ++r) v += f[r] * kap[r * g.nnodes + o];
    return v;
  };
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < g.npts; i += long(gridDim.x) * kBlock) {
    const int jx = int(i % n) + 1, jy = int((i / n) % n) + 1, jz = int(i / (long(n) * n)) + 1;
    const TC kc = node(jx, jy, jz);
    TC d = TC(6) * kc;
    d += node(jx - 1, jy, jz);
    d += node(jx + 1, jy, jz);
    d += node(jx, jy - 1, jz);
    d += node(jx, jy + 1, jz);
    d += node(jx, jy, jz - 1);
    d += node(jx, jy, jz + 1);
    kf[i] = kc;
    df[i] = d;
  }
}

// The wave's pencil: slab s, coarse nodes I0 .. I0 + CX - 1 along x (CX <= 30),
// J0 .. J0 + Jc - 1 along y (Jc <= TY) and K0 .. K0 + Kc - 1 along z; lane l
// holds the fine nodes x = 2 I0 - 2 + l.  False when the wave has no slab or
// its problem has stopped.
struct PencilPos {
  int s, lane, I0, CX, J0, Jc, K0, Kc;
};

template <int TY>
__device__ __forceinline__ bool pencil_pos(const TileJob& J, int pass, PencilPos& P) {
  const int S = J.op.S;
  const int ng = (S + kPencilSlabs - 1) / kPencilSlabs;
  const int lb = int(block_id() - J.block0);
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  P.lane = int(threadIdx.x) & 63;
  const int nc = J.gc.n;
  const int nyt = (nc + TY - 1) / TY, nxs = (nc + kPencilCX - 1) / kPencilCX;
  const int grp = kPencilGroupFastest ? lb % ng : lb / J.tiles;
  int t = kPencilGroupFastest ? lb / ng : lb % J.tiles;
  P.s = grp * kPencilSlabs + pass * kPencilWaves + wave;
  if (P.s >= S) return false;
  if (J.state && done_flag(J.state)) return false;
  int xs, yt;
  if (kPencilXFastest) {
    xs = t % nxs;
    t /= nxs;
    yt = t % nyt;
  } else {
    yt = t % nyt;
    t /= nyt;
    xs = t % nxs;
  }
  const int zt = t / (kPencilXFastest ? nyt : nxs);
  const int cb = nc / nxs, cr = nc % nxs;
  P.I0 = 1 + xs * cb + min(xs, cr);
  P.CX = cb + (xs < cr ? 1 : 0);
  P.J0 = 1 + yt * TY;
  P.K0 = 1 + zt * kPencilTZ;
  P.Jc = min(TY, nc - P.J0 + 1);
  P.Kc = min(kPencilTZ, nc - P.K0 + 1);
  return true;
}

// x1 = omega D^{-1} b and r = b - L x1 on the fine level, r restricted by full
// weighting; one wave per (pencil, slab).  Fine row t of a lane is node y =
// 2 J0 - 2 + t (t = 0 .. 2 TY + 2), plane p is z = 2 K0 - 2 + p.
template <typename TS, typename TC, int TY>
__device__ __forceinline__ void mg_down_pencil(const TileJob& J, const PencilPos& P, TC omega) {
  constexpr int NR = 2 * TY + 3;   // rows of x1, b, k and d
  constexpr int RR = 2 * TY + 1;   // rows of r (t = 1 .. RR)
  const LevelOp L = J.op;
  const int s = P.s, lane = P.lane, I0 = P.I0, CX = P.CX, J0 = P.J0, Jc = P.Jc, K0 = P.K0, Kc = P.Kc;
  const int nf = J.gf.n, nc = J.gc.n;
  const int x = 2 * I0 - 2 + lane;
  const bool xin = unsigned(x - 1) < unsigned(nf);
  const unsigned vS = xin ? unsigned(x - 1) * unsigned(sizeof(TS)) : 0x80000000u;
  const unsigned vC = xin ? unsigned(x - 1) * unsigned(sizeof(TC)) : 0x80000000u;
  const long npf = J.gf.npts;
  const rsrc_t rb = make_rsrc((const TS*)J.b + long(s) * npf, unsigned(npf * long(sizeof(TS))));
  const rsrc_t rk = make_rsrc(J.pk, unsigned(npf * long(sizeof(TC))));
  const rsrc_t rd = make_rsrc(J.pd, unsigned(npf * long(sizeof(TC))));
  const TC* sg = (const TC*)L.sig;
  const TC sigma = sg ? sg[s] : TC(0);
  const TC gamma = slab_scale<TC>(L, s);
  const TC one_m_omega = TC(1) - omega;
  const int yb = 2 * J0 - 2, zb = 2 * K0 - 2;
  TS* bcs = (TS*)J.out + long(s) * J.gc.npts;

  // Rows and planes outside the domain are clamped into it for the loads (so no
  // load is skipped and no branch is taken); x1 is zero there.  A clamped k or b
  // only ever meets x1 = 0 or feeds r at nodes whose coarse node is not stored.
  unsigned roff[NR];
  bool rok[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int y = yb + r;
    rok[r] = unsigned(y - 1) < unsigned(nf);
    roff[r] = unsigned(min(max(y, 1), nf) - 1) * unsigned(nf);
  }
  const unsigned nf2 = unsigned(nf) * unsigned(nf);
  auto load_plane = [&](int q, TC(&b)[NR], TC(&k)[NR], TC(&d)[NR]) {
    const unsigned po = unsigned(min(max(zb + q, 1), nf) - 1) * nf2;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const unsigned row = po + roff[r];
      b[r] = bload<TC, TS>(rb, vS, row * unsigned(sizeof(TS)));
      k[r] = bload<TC, TC>(rk, vC, row * unsigned(sizeof(TC)));
      d[r] = bload<TC, TC>(rd, vC, row * unsigned(sizeof(TC)));
    }
  };
  auto x1_plane = [&](int q, const TC(&b)[NR], const TC(&d)[NR], TC(&xo)[NR]) {
    const bool zok = unsigned(zb + q - 1) < unsigned(nf);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const TC v = omega * b[r] * rcp_fast(sigma + gamma * d[r]);
      xo[r] = (zok && rok[r] && xin) ? v : TC(0);
    }
  };

  // The residual of plane p is summed as the march reaches its terms: when x1
  // of plane p is known, R(p) = (1 - omega) b + gamma (x-, x+, y-, y+, z- face
  // terms); the z+ term completes it once x1 of plane p + 1 is known.  Only
  // R(p), k(p) and x1(p) (Kp, Xp) cross a plane step, plus the kPencilDepth
  // loaded planes ahead (slot q % kPencilDepth): each is issued kPencilDepth
  // steps before its use.
  auto inplane = [&](const TC(&xc)[NR], const TC(&kc)[NR], const TC(&xm)[NR], const TC(&km)[NR],
                     const TC(&bc)[NR], TC(&R)[RR]) {
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      const int r = i + 1;
      const TC c = kc[r];
      TC o = (c + lane_shift<kDppFromLower>(c)) * lane_shift<kDppFromLower>(xc[r]);
      o += (c + lane_shift<kDppFromUpper>(c)) * lane_shift<kDppFromUpper>(xc[r]);
      o += (c + kc[r - 1]) * xc[r - 1];
      o += (c + kc[r + 1]) * xc[r + 1];
      o += (c + km[r]) * xm[r];
      R[i] = one_m_omega * bc[r] + gamma * o;
    }
  };
  constexpr int PD = kPencilDepth;
  TC Bq[PD][NR], Kq[PD][NR], Dq[PD][NR];   // loaded planes, slot q % PD
  TC R[RR], Kp[NR], Xp[NR];
  {
    TC b0[NR], k0[NR], d0[NR], x0[NR], b1[NR], k1[NR], d1[NR];
    load_plane(0, b0, k0, d0);
    load_plane(1, b1, k1, d1);
    x1_plane(0, b0, d0, x0);
    x1_plane(1, b1, d1, Xp);
    inplane(Xp, k1, x0, k0, b1, R);
#pragma unroll
    for (int r = 0; r < NR; ++r) Kp[r] = k1[r];
  }
  const int pend = 2 * Kc + 1;   // r planes p = 1 .. pend
  load_plane(2, Bq[0], Kq[0], Dq[0]);
  if (PD == 2) load_plane(3, Bq[PD - 1], Kq[PD - 1], Dq[PD - 1]);
  TC A[RR];
#pragma unroll
  for (int i = 0; i < RR; ++i) A[i] = TC(0);
  const bool st_lane = (lane & 1) == 0 && lane >= 2 && lane <= 2 * CX;
  const int I = I0 + ((lane - 2) >> 1);

  // r plane p = p0 + u (p0 odd): plane p + 1 sits in slot (p + 1) % PD = u % PD
  auto step = [&](auto U, int p0) -> bool {
    constexpr int u = decltype(U)::value;
    const int p = p0 + u;
    if (p > pend) return false;
    TC(&bn)[NR] = Bq[u % PD];
    TC(&kn)[NR] = Kq[u % PD];
    TC(&dn)[NR] = Dq[u % PD];
    TC xn[NR];
    x1_plane(p + 1, bn, dn, xn);
    TC rv[RR];
#pragma unroll
    for (int i = 0; i < RR; ++i) rv[i] = R[i] + gamma * ((Kp[i + 1] + kn[i + 1]) * xn[i + 1]);
    if (p < pend) {
      inplane(xn, kn, Xp, Kp, bn, R);   // R of plane p + 1
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        Kp[r] = kn[r];
        Xp[r] = xn[r];
      }
      if (p + PD <= pend) load_plane(p + 1 + PD, bn, kn, dn);   // the slot just consumed
    }
    if constexpr (u % 2 == 0) {
      // odd p = 2k + 1 closes coarse plane k - 1 (weight 1/4) and opens plane k
      TC T[RR];
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        T[i] = A[i] + TC(0.25) * rv[i];
        A[i] = TC(0.25) * rv[i];
      }
      if (p >= 3) {
        const int K = K0 + ((p - 3) >> 1);
#pragma unroll
        for (int j = 0; j < TY; ++j) {
          const TC Y = TC(0.25) * T[2 * j] + TC(0.5) * T[2 * j + 1] + TC(0.25) * T[2 * j + 2];
          const TC X = TC(0.25) * lane_shift<kDppFromLower>(Y) + TC(0.5) * Y + TC(0.25) * lane_shift<kDppFromUpper>(Y);
          if (st_lane && j < Jc) st<TS, TC>(bcs, (long(K - 1) * nc + (J0 + j - 1)) * nc + (I - 1), X);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < RR; ++i) A[i] += TC(0.5) * rv[i];
    }
    return true;
  };
  for (int p0 = 1; p0 <= pend; p0 += 2) {
    if (!step(std::integral_constant<int, 0>{}, p0)) break;
    if (!step(std::integral_constant<int, 1>{}, p0)) break;
  }
}

template <typename TS, typename TC, int TY>
__global__ void __launch_bounds__(kPencilThreads) k_mg_down_p3(const TileJob* __restrict__ jobs, int njobs, TC omega) {
  const TileJob J = to_global(jobs[find_job(jobs, njobs)]);
  for (int pass = 0; pass < kPencilPasses; ++pass) {
    PencilPos P;
    if (!pencil_pos<TY>(J, pass, P)) return;
    mg_down_pencil<TS, TC, TY>(J, P, omega);
  }
}

// x2 = omega D^{-1} b + P e and x = (1 - omega) x2 + omega D^{-1} (b + gamma
// sum_nb w x2_nb) on the fine level (P: multilinear prolongation of the
// coarse correction e), one wave per (pencil, slab) as in the down-sweep.  A
// wave writes the fine nodes 2I - 1 and 2I of its coarse nodes I (and node n
// when its pencil ends the axis); x2 is needed one node further.  Epilogue:
// store x (EPI_STORE), add it into the output (EPI_ADDTS) or into the float64 acc64 (EPI_ADD64).
// The arithmetic per fine node is that of the tiled kernel.
template <typename TS, typename TC, int TY, int EPI>
__device__ __forceinline__ void mg_up_pencil(const TileJob& J, const PencilPos& P, TC omega) {
  constexpr int NR = 2 * TY + 3;   // fine rows t = 0 .. NR - 1 (node y = 2 J0 - 2 + t)
  constexpr int RR = 2 * TY + 1;   // rows that can be written (t = 1 .. RR)
  constexpr int NE = TY + 2;       // coarse rows J0 - 1 .. J0 + TY of e
  const LevelOp L = J.op;
  const int s = P.s, lane = P.lane, I0 = P.I0, CX = P.CX, J0 = P.J0, Jc = P.Jc, K0 = P.K0, Kc = P.Kc;
  const int nf = J.gf.n, nc = J.gc.n;
  const int x = 2 * I0 - 2 + lane;
  const bool xin = unsigned(x - 1) < unsigned(nf);
  const unsigned vS = xin ? unsigned(x - 1) * unsigned(sizeof(TS)) : 0x80000000u;
  const unsigned vC = xin ? unsigned(x - 1) * unsigned(sizeof(TC)) : 0x80000000u;
  const int Ie = I0 - 1 + (lane >> 1);   // coarse node of e this lane loads
  const unsigned vE = unsigned(Ie - 1) < unsigned(nc) ? unsigned(Ie - 1) * unsigned(sizeof(TS)) : 0x80000000u;
  const bool lastx = I0 + CX - 1 == nc, lasty = J0 + Jc - 1 == nc, lastz = K0 + Kc - 1 == nc;
  const bool outx = (lane >= 1 && lane <= 2 * CX) || (lastx && lane == 2 * CX + 1);
  const long npf = J.gf.npts, npc = J.gc.npts;
  const rsrc_t rb = make_rsrc((const TS*)J.b + long(s) * npf, unsigned(npf * long(sizeof(TS))));
  const rsrc_t re = make_rsrc((const TS*)J.e + long(s) * npc, unsigned(npc * long(sizeof(TS))));
  const rsrc_t rk = make_rsrc(J.pk, unsigned(npf * long(sizeof(TC))));
  const rsrc_t rd = make_rsrc(J.pd, unsigned(npf * long(sizeof(TC))));
  const TC* sg = (const TC*)L.sig;
  const TC sigma = sg ? sg[s] : TC(0);
  const TC gamma = slab_scale<TC>(L, s);
  const TC one_m_omega = TC(1) - omega;
  const int yb = 2 * J0 - 2, zb = 2 * K0 - 2;
  TS* os = (TS*)J.out + long(s) * npf;
  double* as = J.acc64 + long(s) * npf;

  unsigned roff[NR];
  bool rok[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int y = yb + r;
    rok[r] = unsigned(y - 1) < unsigned(nf);
    roff[r] = unsigned(min(max(y, 1), nf) - 1) * unsigned(nf);
  }
  const unsigned nf2 = unsigned(nf) * unsigned(nf), nc2 = unsigned(nc) * unsigned(nc);
  auto load_plane = [&](int q, TC(&b)[NR], TC(&k)[NR], TC(&d)[NR]) {
    const unsigned po = unsigned(min(max(zb + q, 1), nf) - 1) * nf2;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const unsigned row = po + roff[r];
      b[r] = bload<TC, TS>(rb, vS, row * unsigned(sizeof(TS)));
      k[r] = bload<TC, TC>(rk, vC, row * unsigned(sizeof(TC)));
      d[r] = bload<TC, TC>(rd, vC, row * unsigned(sizeof(TC)));
    }
  };
  // coarse plane c of e (node K0 - 1 + c), rows J0 - 1 .. J0 + TY; zero outside the coarse interior
  auto load_e = [&](int c, TC(&er)[NE]) {
    const int Kz = K0 - 1 + c;
    const bool zok = unsigned(Kz - 1) < unsigned(nc);
    const unsigned po = unsigned(min(max(Kz, 1), nc) - 1) * nc2;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int Jy = J0 - 1 + j;
      const bool ok = zok && unsigned(Jy - 1) < unsigned(nc);
      const unsigned row = po + unsigned(min(max(Jy, 1), nc) - 1) * unsigned(nc);
      er[j] = bload<TC, TS>(re, ok ? vE : 0x80000000u, row * unsigned(sizeof(TS)));
    }
  };
  // e interpolated along x, then y, onto the fine rows of the lane
  auto pxy_plane = [&](const TC(&er)[NE], TC(&pv)[NR]) {
    TC ex[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const TC nx = lane_shift<kDppFromUpper>(er[j]);
      ex[j] = (lane & 1) ? TC(0.5) * (er[j] + nx) : er[j];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) pv[r] = (r & 1) ? TC(0.5) * (ex[r >> 1] + ex[(r >> 1) + 1]) : ex[r >> 1];
  };
  // x2 and omega D^{-1} of fine plane q from its b, d and the interpolated e
  auto x2_plane = [&](int q, const TC(&b)[NR], const TC(&d)[NR], const TC(&pe)[NR], TC(&xo)[NR], TC(&wo)[NR]) {
    const bool zok = unsigned(zb + q - 1) < unsigned(nf);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const TC wd = omega * rcp_fast(sigma + gamma * d[r]);
      wo[r] = wd;
      xo[r] = (zok && rok[r] && xin) ? wd * b[r] + pe[r] : TC(0);
    }
  };

  // Streaming as in the down-sweep: the smoothing sum of plane p gets its x-,
  // x+, y-, y+ and z- terms when x2 of plane p is known (O5) and its z+ term
  // with x2 of plane p + 1.  Across a plane step: x2(p), k(p), O5(p), omega
  // D^{-1} and b of plane p, the loaded planes p + 1, p + 2 (slot q % 2), the
  // interpolated e of two coarse planes (slot c % 2) and the raw e of the next.
  auto inplane = [&](const TC(&xc)[NR], const TC(&kc)[NR], const TC(&xm)[NR], const TC(&km)[NR], TC(&O)[RR]) {
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      const int r = i + 1;
      const TC c = kc[r];
      TC o = (c + lane_shift<kDppFromLower>(c)) * lane_shift<kDppFromLower>(xc[r]);
      o += (c + lane_shift<kDppFromUpper>(c)) * lane_shift<kDppFromUpper>(xc[r]);
      o += (c + kc[r - 1]) * xc[r - 1];
      o += (c + kc[r + 1]) * xc[r + 1];
      o += (c + km[r]) * xm[r];
      O[i] = o;
    }
  };
  const int pend = 2 * Kc + 1;   // planes p = 1 .. pend (the last one written only at the end of the axis)
  const int rlast = lasty ? 2 * Jc + 1 : 2 * Jc;   // rows written: 1 .. rlast
  const int plast = lastz ? pend : pend - 1;      // planes written: 1 .. plast
  // output (or float64 target) rows of plane q, read ahead for the epilogues that add
  auto load_acc = [&](int q, double(&a)[RR]) {
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      a[i] = 0.0;
      const int r = i + 1;
      if (q <= plast && r <= rlast && outx) {
        const long o = long(zb + q - 1) * nf2 + long(yb + r - 1) * nf + (x - 1);
        if (EPI == EPI_ADD64) a[i] = as[o];
        else if (EPI == EPI_ADDTS) a[i] = double(ld<TC>(os, o));
      }
    }
  };
  TC Bq[2][NR], Kq[2][NR], Dq[2][NR], Pp[2][NR], ER[NE];
  TC X2p[NR], Kp[NR], O5[RR], WD[RR], BB[RR];
  double AC[RR];
  {
    TC b0[NR], k0[NR], d0[NR], x0[NR], w0[NR], w1[NR], pe[NR];
    load_plane(0, b0, k0, d0);
    load_plane(1, Bq[1], Kq[1], Dq[1]);
    TC e0[NE];
    load_e(0, e0);
    load_e(1, ER);
    pxy_plane(e0, Pp[0]);
    pxy_plane(ER, Pp[1]);
    load_e(2, ER);
    x2_plane(0, b0, d0, Pp[0], x0, w0);
#pragma unroll
    for (int r = 0; r < NR; ++r) pe[r] = TC(0.5) * (Pp[0][r] + Pp[1][r]);
    x2_plane(1, Bq[1], Dq[1], pe, X2p, w1);
    inplane(X2p, Kq[1], x0, k0, O5);
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      WD[i] = w1[i + 1];
      BB[i] = Bq[1][i + 1];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) Kp[r] = Kq[1][r];
  }
  load_plane(2, Bq[0], Kq[0], Dq[0]);
  load_plane(3, Bq[1], Kq[1], Dq[1]);
  if (EPI != EPI_STORE) load_acc(1, AC);

  // plane p = p0 + u (p0 odd): writes plane p, computes x2 of plane q = p + 1
  // (slot q % 2 = u % 2; q even for even u, coarse plane c = q / 2)
  auto step = [&](auto U, int p0) -> bool {
    constexpr int u = decltype(U)::value;
    const int p = p0 + u;
    if (p > pend) return false;
    TC(&bn)[NR] = Bq[u % 2];
    TC(&kn)[NR] = Kq[u % 2];
    TC(&dn)[NR] = Dq[u % 2];
    TC xn[NR], wn[NR];
    if constexpr (u % 2 == 0) {
      // q = 2c: coarse plane c is in slot c % 2 = ((p + 1) / 2) % 2; c + 1 goes to the other slot
      const int c = (p + 1) >> 1;
      if (c & 1) {
        pxy_plane(ER, Pp[0]);
        x2_plane(p + 1, bn, dn, Pp[1], xn, wn);
      } else {
        pxy_plane(ER, Pp[1]);
        x2_plane(p + 1, bn, dn, Pp[0], xn, wn);
      }
      load_e(c + 2, ER);
    } else {
      TC pe[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) pe[r] = TC(0.5) * (Pp[0][r] + Pp[1][r]);
      x2_plane(p + 1, bn, dn, pe, xn, wn);
    }
    if (p <= plast) {
      const long po = long(zb + p - 1) * nf2;
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        const int r = i + 1;
        TC off = O5[i] + (Kp[r] + kn[r]) * xn[r];
        off *= gamma;
        const TC v = one_m_omega * X2p[r] + WD[i] * (BB[i] + off);
        if (r <= rlast && outx) {
          const long o = po + long(yb + r - 1) * nf + (x - 1);
          if (EPI == EPI_ADD64) as[o] = AC[i] + double(v);
          else st<TS, TC>(os, o, EPI == EPI_ADDTS ? TC(AC[i]) + v : v);
        }
      }
    }
    if (p < pend) {
      inplane(xn, kn, X2p, Kp, O5);
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        WD[i] = wn[i + 1];
        BB[i] = bn[i + 1];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        X2p[r] = xn[r];
        Kp[r] = kn[r];
      }
      if (p + 2 <= pend) load_plane(p + 3, bn, kn, dn);
      if (EPI != EPI_STORE) load_acc(p + 1, AC);
    }
    return true;
  };
  for (int p0 = 1; p0 <= pend; p0 += 2) {
    if (!step(std::integral_constant<int, 0>{}, p0)) break;
    if (!step(std::integral_constant<int, 1>{}, p0)) break;
  }
}

template <typename TS, typename TC, int TY, int EPI>
__global__ void __launch_bounds__(kPencilThreads) k_mg_up_p3(const TileJob* __restrict__ jobs, int njobs, TC omega) {
  const TileJob J = to_global(jobs[find_job(jobs, njobs)]);
  for (int pass = 0; pass < kPencilPasses; ++pass) {
    PencilPos P;
    if (!pencil_pos<TY>(J, pass, P)) return;
    mg_up_pencil<TS, TC, TY, EPI>(J, P, omega);
  }
}

}  // namespace stp

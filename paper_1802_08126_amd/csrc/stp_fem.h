// Kernels of the finite-element discretisation: a general (here: consistent
// finite-element) mass matrix M in K = bidiag (x) M and in H_k = mu_k M +
// tau A (Section 2, eqs. (2.3)-(2.5), (4.5)), for the elements of the paper's
// experiments on uniform meshes of the unit d-cube: P1 in 1-D and 2-D (every
// square split by its lower-left/upper-right diagonal), Q1 in 3-D, with a
// coefficient constant in space (a factor a(t_n) of the stiffness).
//
// Every operator of a level is sigma_s M + c_s A with M and A the same
// 3^d-point stencil at every node, so the kernels read the two weight sets
// from their arguments and the vectors through the caches; one thread owns
// one node of one slab.  Multigrid levels use the Galerkin operators of the
// finite-element interpolation P (trilinear, or P1-linear in 2-D) with
// R = P^T / 2^d, which are the element operators of the coarse meshes scaled
// by 2^-d per level; the weights passed in already carry that scaling.
#pragma once
#include "stp_kernels.h"

namespace stp {

// Stencil weights of M and A on one level: neighbour (dx, dy, dz) in
// {-1,0,1}^d has index ((dz+1)*3 + (dy+1))*3 + (dx+1) (dz = 0 in 2-D,
// dy = dz = 0 in 1-D); index 13 (3-D), 4 (2-D), 1 (1-D) is the node itself.
template <typename TC>
struct FemW {
  TC m[27];
  TC a[27];
};

template <int D>
__host__ __device__ constexpr int fem_nb() { return D == 1 ? 3 : (D == 2 ? 9 : 27); }
template <int D>
__host__ __device__ constexpr int fem_ctr() { return D == 1 ? 1 : (D == 2 ? 4 : 13); }

// the vectors of the current solve, read when a kernel runs (so captured
// graphs follow a rebinding): u, p, the source F and u0, the float64 target of
// the A-tilde solve
struct FemBind {
  const double* u;
  const double* p;
  const double* F;
  const double* u0;
  double* accp;
};

__device__ __forceinline__ FemBind to_global(FemBind b) {
  b.u = gmem(b.u);
  b.p = gmem(b.p);
  b.F = gmem(b.F);
  b.u0 = gmem(b.u0);
  b.accp = gmem(b.accp);
  return b;
}

// Calls f(k, j) for every neighbour k of interior node (x, y, z) (0-based)
// that is an interior node, j its offset inside the slab.
template <int D, typename Fn>
__device__ __forceinline__ void fem_for_nb(int x, int y, int z, int n, Fn&& f) {
#pragma unroll
  for (int k = 0; k < fem_nb<D>(); ++k) {
    const int dx = k % 3 - 1;
    const int dy = D >= 2 ? (k / 3) % 3 - 1 : 0;
    const int dz = D >= 3 ? k / 9 - 1 : 0;
    const int X = x + dx, Y = y + dy, Z = z + dz;
    bool ok = unsigned(X) < unsigned(n);
    if (D >= 2) ok = ok && unsigned(Y) < unsigned(n);
    if (D >= 3) ok = ok && unsigned(Z) < unsigned(n);
    if (ok) f(k, D == 1 ? X : (D == 2 ? Y * n + X : (Z * n + Y) * n + X));
  }
}

// slab operator (sigma_s, c_s): sig may be null (sigma = 0); cstride 0 means
// one c for every slab
template <typename TC>
__device__ __forceinline__ void fem_op(const TC* sig, const TC* c, int cstride, int s, TC& sg, TC& cc) {
  sg = sig ? sig[s] : TC(0);
  cc = c[long(s) * cstride];
}

// ---------------------------------------------------------------------------
// outer residuals (float64), eq. (3.1) with K = bidiag (x) M:
//   a1: r_p = M (u_n - u_{n-1} - tau_n F_n - [n=1] u0) - c_n A p_n
//   a3: r_u = M (tau_n F_n + [n=1] u0 - (p_n - p_{n+1}) - (2u_n - u_{n-1} - u_{n+1})) - c_n A u_n
//       and partials of ||f - B u||^2, (f - B u)_n = M (tau_n F_n + [n=1] u0 - (u_n - u_{n-1})) - c_n A u_n
// c_n = tau_n a_n (cA, stride kMaxRank).  Grid: grid_pts(npts, N).
// ---------------------------------------------------------------------------
template <int D, typename TS, int WHICH>
__global__ void __launch_bounds__(kBlock) k_fem_resid(Geom g, int N, FemW<double> w, const double* __restrict__ taus,
                                                      const double* __restrict__ cA, const FemBind* __restrict__ fb,
                                                      const int* __restrict__ state, TS* __restrict__ r,
                                                      double* __restrict__ partial) {
  if (done_flag(state)) return;
  const FemBind B = to_global(*fb);
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double e2 = 0.0;
  if (s < N && i < g.npts) {
    int x, y, z;
    decode<D>(i, g.n, x, y, z);
    const long np = g.npts, o = long(s) * np;
    const double ts = taus[s], cn = cA[long(s) * kMaxRank];
    const bool first = s == 0, last = s + 1 == N;
    double mv = 0.0, av = 0.0, me = 0.0;
    fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) {
      const double uc = B.u[o + j];
      const double um = first ? 0.0 : B.u[o - np + j];
      const double fj = ts * B.F[o + j] + (first ? B.u0[j] : 0.0);
      if (WHICH == 0) {
        mv += w.m[k] * (uc - um - fj);
        av += w.a[k] * B.p[o + j];
      } else {
        const double up = last ? 0.0 : B.u[o + np + j];
        const double pp = last ? 0.0 : B.p[o + np + j];
        mv += w.m[k] * (fj - (B.p[o + j] - pp) - (2.0 * uc - um - up));
        me += w.m[k] * (fj - (uc - um));
        av += w.a[k] * uc;
      }
    });
    st<TS, double>(r, o + i, mv - cn * av);
    if (WHICH == 1) {
      const double e = me - cn * av;
      e2 = e * e;
    }
  }
  if (WHICH == 1) {
    const double bs = block_sum(e2);
    if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
  }
}

// ---------------------------------------------------------------------------
// multigrid V-cycle on sigma_s M + c_s A (Galerkin levels) with s sweeps of
// damped l1-Jacobi before and after the coarse correction:
//   x <- x + theta (b - L x) / l1,   l1 = sum over the stencil of |sigma m_k + c a_k|,
// the absolute row sum of L (a Gershgorin bound of lambda_max(D^{-1} L) times the
// diagonal, which is the same at every node), so theta < 2 contracts every
// sweep whatever the mix of mass and stiffness.
// ---------------------------------------------------------------------------
template <int D, typename TC>
__device__ __forceinline__ TC fem_l1(const FemW<TC>& w, TC sg, TC cc) {
  TC a = 0;
#pragma unroll
  for (int k = 0; k < fem_nb<D>(); ++k) a += fabs(sg * w.m[k] + cc * w.a[k]);
  return a;
}

// first sweep from the zero guess: x = (theta / l1) b
template <int D, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_fem_jac0(long npts, int S, FemW<TC> w, const TC* __restrict__ sig,
                                                     const TC* __restrict__ c, int cstride, TC theta,
                                                     const TS* __restrict__ b, TS* __restrict__ x,
                                                     const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || i >= npts) return;
  TC sg, cc;
  fem_op(sig, c, cstride, s, sg, cc);
  const long o = long(s) * npts + i;
  st<TS, TC>(x, o, (theta / fem_l1<D, TC>(w, sg, cc)) * ld<TC>(b, o));
}

// one sweep v = x + (theta / l1) (b - L x): stored (TS), or (EPI_ADD64) added
// into the binding's float64 target (the A-tilde solve into p)
template <int D, typename TS, typename TC, int EPI>
__global__ void __launch_bounds__(kBlock) k_fem_sweep(Geom g, int S, FemW<TC> w, const TC* __restrict__ sig,
                                                      const TC* __restrict__ c, int cstride, TC theta,
                                                      const TS* __restrict__ b, const TS* __restrict__ xv,
                                                      TS* __restrict__ out, const FemBind* __restrict__ fb,
                                                      const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || i >= g.npts) return;
  int x, y, z;
  decode<D>(i, g.n, x, y, z);
  TC sg, cc;
  fem_op(sig, c, cstride, s, sg, cc);
  const long o = long(s) * g.npts;
  const TS* xs = xv + o;
  TC lx = 0;
  fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) { lx += (sg * w.m[k] + cc * w.a[k]) * ld<TC>(xs, j); });
  const TC v = ld<TC>(xs, i) + (theta / fem_l1<D, TC>(w, sg, cc)) * (ld<TC>(b, o + i) - lx);
  if (EPI == EPI_STORE) {
    st<TS, TC>(out, o + i, v);
  } else {
    double* acc = gmem(fb->accp);
    acc[o + i] += double(v);
  }
}

// residual r = b - L x
template <int D, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_fem_res(Geom g, int S, FemW<TC> w, const TC* __restrict__ sig,
                                                    const TC* __restrict__ c, int cstride, const TS* __restrict__ b,
                                                    const TS* __restrict__ xv, TS* __restrict__ r,
                                                    const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || i >= g.npts) return;
  int x, y, z;
  decode<D>(i, g.n, x, y, z);
  TC sg, cc;
  fem_op(sig, c, cstride, s, sg, cc);
  const long o = long(s) * g.npts;
  const TS* xs = xv + o;
  TC lx = 0;
  fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) { lx += (sg * w.m[k] + cc * w.a[k]) * ld<TC>(xs, j); });
  st<TS, TC>(r, o + i, ld<TC>(b, o + i) - lx);
}

// restriction R = P^T / 2^d: bc_I = sum_o rw(o) r_{2I+o} (fine nodes around
// coarse node I); trilinear: prod_a (1/2 at o_a = 0, 1/4 at +-1); P1 in 2-D:
// 1/4 at the node, 1/8 on its four edges and its lower-left and upper-right
// diagonal neighbours
template <int D, typename TS, typename TC, bool P1>
__global__ void __launch_bounds__(kBlock) k_fem_restrict(Geom gf, Geom gc, int S, const TS* __restrict__ r,
                                                         TS* __restrict__ bc, const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long I = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || I >= gc.npts) return;
  int X, Y, Z;
  decode<D>(I, gc.n, X, Y, Z);
  // coarse node (0-based) X sits at fine node 2X + 1 (0-based)
  const int fx = 2 * X + 1, fy = D >= 2 ? 2 * Y + 1 : 0, fz = D >= 3 ? 2 * Z + 1 : 0;
  const TS* rs = r + long(s) * gf.npts;
  TC acc = 0;
  fem_for_nb<D>(fx, fy, fz, gf.n, [&](int k, int j) {
    const int dx = k % 3 - 1, dy = D >= 2 ? (k / 3) % 3 - 1 : 0, dz = D >= 3 ? k / 9 - 1 : 0;
    TC wt;
    if (P1 && D == 2) {
      wt = (dx == 0 && dy == 0) ? TC(0.25) : (dx == -dy && dx != 0 ? TC(0) : TC(0.125));
    } else {
      wt = (dx == 0 ? TC(0.5) : TC(0.25));
      if (D >= 2) wt *= (dy == 0 ? TC(0.5) : TC(0.25));
      if (D >= 3) wt *= (dz == 0 ? TC(0.5) : TC(0.25));
    }
    acc += wt * ld<TC>(rs, j);
  });
  st<TS, TC>(bc, long(s) * gc.npts + I, acc);
}

// coarse-grid correction x += P e (interpolation of the coarse correction:
// fine node j (1-based) takes coarse j/2 when even, the mean of (j-1)/2 and
// (j+1)/2 when odd; in 2-D P1 a node odd in both takes the mean of the
// lower-left and upper-right coarse corners)
template <int D, typename TS, typename TC, bool P1>
__global__ void __launch_bounds__(kBlock) k_fem_prolong_add(Geom gf, Geom gc, int S, const TS* __restrict__ e,
                                                            TS* __restrict__ xv, const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || i >= gf.npts) return;
  int x, y, z;
  decode<D>(i, gf.n, x, y, z);
  const TS* es = e + long(s) * gc.npts;
  const int nc = gc.n;
  // coarse value at 1-based coarse node (X, Y, Z), zero on the boundary
  auto ec = [&](int X, int Y, int Z) -> TC {
    bool ok = X >= 1 && X <= nc;
    if (D >= 2) ok = ok && Y >= 1 && Y <= nc;
    if (D >= 3) ok = ok && Z >= 1 && Z <= nc;
    if (!ok) return TC(0);
    const int q = D == 1 ? X - 1 : (D == 2 ? (Y - 1) * nc + X - 1 : ((Z - 1) * nc + Y - 1) * nc + X - 1);
    return ld<TC>(es, q);
  };
  const int jx = x + 1, jy = D >= 2 ? y + 1 : 0, jz = D >= 3 ? z + 1 : 0;   // 1-based fine node
  TC pe = 0;
  if (P1 && D == 2 && (jx & 1) && (jy & 1)) {
    pe = TC(0.5) * (ec(jx >> 1, jy >> 1, 0) + ec((jx >> 1) + 1, (jy >> 1) + 1, 0));
  } else {
    const int lx = jx >> 1, ly = jy >> 1, lz = jz >> 1;
    const int ox = jx & 1, oy = D >= 2 ? (jy & 1) : 0, oz = D >= 3 ? (jz & 1) : 0;
#pragma unroll
    for (int cz = 0; cz <= (D >= 3 ? 1 : 0); ++cz)
#pragma unroll
      for (int cy = 0; cy <= (D >= 2 ? 1 : 0); ++cy)
#pragma unroll
        for (int cx = 0; cx <= 1; ++cx) {
          if ((cx && !ox) || (cy && !oy) || (cz && !oz)) continue;
          TC wt = ox ? TC(0.5) : TC(1);
          if (D >= 2) wt *= oy ? TC(0.5) : TC(1);
          if (D >= 3) wt *= oz ? TC(0.5) : TC(1);
          pe += wt * ec(lx + cx, ly + cy, lz + cz);
        }
  }
  const long o = long(s) * gf.npts + i;
  st<TS, TC>(xv, o, ld<TC>(xv, o) + pe);
}

// one-node level: e = b / (sigma m_c + c a_c)
template <typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_fem_coarsest(int S, TC mc, TC ac, const TC* __restrict__ sig,
                                                         const TC* __restrict__ c, int cstride,
                                                         const TS* __restrict__ b, TS* __restrict__ e,
                                                         const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = int(long(blockIdx.x) * kBlock + threadIdx.x);
  if (s >= S) return;
  TC sg, cc;
  fem_op(sig, c, cstride, s, sg, cc);
  st<TS, TC>(e, s, ld<TC>(b, s) / (sg * mc + cc * ac));
}

// the middle operator of the H-blocks: y = cmid A x
template <int D, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock) k_fem_apply(Geom g, int S, FemW<TC> w, TC cmid, const TS* __restrict__ xv,
                                                      TS* __restrict__ y, const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= S || i >= g.npts) return;
  int x, yy, z;
  decode<D>(i, g.n, x, yy, z);
  const TS* xs = xv + long(s) * g.npts;
  TC ax = 0;
  fem_for_nb<D>(x, yy, z, g.n, [&](int k, int j) { ax += w.a[k] * ld<TC>(xs, j); });
  st<TS, TC>(y, long(s) * g.npts + i, cmid * ax);
}

// exact 1-D solves of (sigma_s M + c_s A) x = b (constant bands), one thread
// per slab (Thomas algorithm; scratch: S x n values); EPI_ADD64 adds into the
// binding's float64 target
template <typename TS, typename TC, int EPI>
__global__ void __launch_bounds__(64) k_fem_tridiag(int n, int S, TC m0, TC m1, TC a0, TC a1,
                                                    const TC* __restrict__ sig, const TC* __restrict__ c, int cstride,
                                                    const TS* __restrict__ b, TS* __restrict__ out,
                                                    const FemBind* __restrict__ fb, TC* __restrict__ scratch,
                                                    const int* __restrict__ state) {
  if (done_flag(state)) return;
  const int s = int(long(blockIdx.x) * 64 + threadIdx.x);
  if (s >= S) return;
  TC sg, cc;
  fem_op(sig, c, cstride, s, sg, cc);
  const TC dd = sg * m0 + cc * a0, oo = sg * m1 + cc * a1;
  const long o = long(s) * n;
  TC* cp = scratch + o;      // modified super-diagonal, then the solution in place of d'
  const TS* bs = b + o;
  // forward sweep: cp_i = oo / (dd - oo cp_{i-1}), dp_i = (b_i - oo dp_{i-1}) / (dd - oo cp_{i-1})
  TC cprev = 0, dprev = 0;
  for (int i = 0; i < n; ++i) {
    const TC den = dd - oo * cprev;
    cprev = oo / den;
    dprev = (ld<TC>(bs, i) - oo * dprev) / den;
    cp[i] = cprev;
    scratch[long(S) * n + o + i] = dprev;   // d' in the second half of the scratch
  }
  TC xn = 0;
  for (int i = n - 1; i >= 0; --i) {
    const TC v = scratch[long(S) * n + o + i] - cp[i] * xn;
    xn = v;
    if (EPI == EPI_STORE) st<TS, TC>(out, o + i, v);
    else gmem(fb->accp)[o + i] += double(v);
  }
}

// ||f||^2 partials, f_n = M (tau_n F_n + [n=1] u0)
template <int D>
__global__ void __launch_bounds__(kBlock) k_fem_fnorm(Geom g, int N, FemW<double> w, const double* __restrict__ taus,
                                                      const double* __restrict__ F, const double* __restrict__ u0,
                                                      double* __restrict__ partial) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double v = 0.0;
  if (s < N && i < g.npts) {
    int x, y, z;
    decode<D>(i, g.n, x, y, z);
    const long o = long(s) * g.npts;
    double f = 0.0;
    fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) { f += w.m[k] * (taus[s] * F[o + j] + (s == 0 ? u0[j] : 0.0)); });
    v = f * f;
  }
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// time-global operators with M (float64): the saddle matrix of eq. (2.7),
// B = K + A of eq. (2.3), residuals and norms for the Krylov acceleration
// ---------------------------------------------------------------------------
// y_p = A p - K u,  y_u = -K^T p - (K + K^T + A) u   (apply: ADD = false);
// r_p = -f - (A p - K u), r_u = -f + K^T p + (K + K^T + A) u   (residual: RES = true)
template <int D, bool RES>
__global__ void __launch_bounds__(kBlock) k_fem_saddle(Geom g, int N, FemW<double> w, const double* __restrict__ taus,
                                                       const double* __restrict__ cA, const double* __restrict__ F,
                                                       const double* __restrict__ u0, const double* __restrict__ p,
                                                       const double* __restrict__ u, double* __restrict__ yp,
                                                       double* __restrict__ yu) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= N || i >= g.npts) return;
  int x, y, z;
  decode<D>(i, g.n, x, y, z);
  const long np = g.npts, o = long(s) * np;
  const double cn = cA[long(s) * kMaxRank];
  const bool first = s == 0, last = s + 1 == N;
  double ku = 0.0, ktp = 0.0, ksym = 0.0, ap = 0.0, au = 0.0, f = 0.0;
  fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) {
    const double uc = u[o + j], um = first ? 0.0 : u[o - np + j], up = last ? 0.0 : u[o + np + j];
    const double pc = p[o + j], pp = last ? 0.0 : p[o + np + j];
    ku += w.m[k] * (uc - um);
    ktp += w.m[k] * (pc - pp);
    ksym += w.m[k] * (2.0 * uc - um - up);
    ap += w.a[k] * pc;
    au += w.a[k] * uc;
    if (RES) f += w.m[k] * (taus[s] * F[o + j] + (first ? u0[j] : 0.0));
  });
  const double tp = cn * ap - ku;
  const double tu = -ktp - ksym - cn * au;
  if (RES) {
    yp[o + i] = -f - tp;
    yu[o + i] = -f - tu;
  } else {
    yp[o + i] = tp;
    yu[o + i] = tu;
  }
}

// y = B x = K x + A x
template <int D>
__global__ void __launch_bounds__(kBlock) k_fem_apply_B(Geom g, int N, FemW<double> w, const double* __restrict__ cA,
                                                        const double* __restrict__ xv, double* __restrict__ y) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= N || i >= g.npts) return;
  int x, yy, z;
  decode<D>(i, g.n, x, yy, z);
  const long np = g.npts, o = long(s) * np;
  double kx = 0.0, ax = 0.0;
  fem_for_nb<D>(x, yy, z, g.n, [&](int k, int j) {
    kx += w.m[k] * (xv[o + j] - (s > 0 ? xv[o - np + j] : 0.0));
    ax += w.a[k] * xv[o + j];
  });
  y[o + i] = kx + cA[long(s) * kMaxRank] * ax;
}

// partials of ||f - B u||^2 over a (points, slabs) grid
template <int D>
__global__ void __launch_bounds__(kBlock) k_fem_fmBu_partial(Geom g, int N, FemW<double> w,
                                                             const double* __restrict__ taus,
                                                             const double* __restrict__ cA,
                                                             const double* __restrict__ F,
                                                             const double* __restrict__ u0,
                                                             const double* __restrict__ u,
                                                             double* __restrict__ partial) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  double v = 0.0;
  if (s < N && i < g.npts) {
    int x, y, z;
    decode<D>(i, g.n, x, y, z);
    const long np = g.npts, o = long(s) * np;
    double me = 0.0, au = 0.0;
    fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) {
      const double uc = u[o + j], um = s > 0 ? u[o - np + j] : 0.0;
      me += w.m[k] * (taus[s] * F[o + j] + (s == 0 ? u0[j] : 0.0) - (uc - um));
      au += w.a[k] * uc;
    });
    const double e = me - cA[long(s) * kMaxRank] * au;
    v = e * e;
  }
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partial[long(slab_index()) * gridDim.x + blockIdx.x] = bs;
}

// partials of ||r_p||^2 and ||r_u||^2 of a pair (p, u) (fixed grid of G blocks
// striding over the points, each thread walking all slabs); block b writes
// partial[b] and partial[G + b]
template <int D>
__global__ void __launch_bounds__(kBlock) k_fem_saddle_norms(Geom g, int N, FemW<double> w,
                                                             const double* __restrict__ taus,
                                                             const double* __restrict__ cA,
                                                             const double* __restrict__ F,
                                                             const double* __restrict__ u0,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ u,
                                                             double* __restrict__ partial) {
  double vp = 0.0, vu = 0.0;
  for (long i = long(blockIdx.x) * kBlock + threadIdx.x; i < g.npts; i += long(gridDim.x) * kBlock) {
    int x, y, z;
    decode<D>(i, g.n, x, y, z);
    for (int s = 0; s < N; ++s) {
      const long np = g.npts, o = long(s) * np;
      const double cn = cA[long(s) * kMaxRank];
      const bool first = s == 0, last = s + 1 == N;
      double ku = 0.0, ktp = 0.0, ksym = 0.0, ap = 0.0, au = 0.0, f = 0.0;
      fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) {
        const double uc = u[o + j], um = first ? 0.0 : u[o - np + j], up = last ? 0.0 : u[o + np + j];
        const double pc = p[o + j], pp = last ? 0.0 : p[o + np + j];
        ku += w.m[k] * (uc - um);
        ktp += w.m[k] * (pc - pp);
        ksym += w.m[k] * (2.0 * uc - um - up);
        ap += w.a[k] * pc;
        au += w.a[k] * uc;
        f += w.m[k] * (taus[s] * F[o + j] + (first ? u0[j] : 0.0));
      });
      const double rp = ku - cn * ap - f;
      const double ru = f - ktp - ksym - cn * au;
      vp += rp * rp;
      vu += ru * ru;
    }
  }
  const double sp = block_sum(vp);
  if (threadIdx.x == 0) partial[blockIdx.x] = sp;
  __syncthreads();   // block_sum's LDS slots are reused
  const double su = block_sum(vu);
  if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = su;
}

// out = sgn (r + K^T d) = sgn (r_n + M (d_n - d_{n+1})), in the storage type
template <int D, typename TS>
__global__ void __launch_bounds__(kBlock) k_fem_kt_add_cast(Geom g, int N, FemW<double> w,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ d, double sgn,
                                                            TS* __restrict__ out) {
  const int s = slab_index();
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= N || i >= g.npts) return;
  int x, y, z;
  decode<D>(i, g.n, x, y, z);
  const long np = g.npts, o = long(s) * np;
  double v = 0.0;
  fem_for_nb<D>(x, y, z, g.n, [&](int k, int j) { v += w.m[k] * (d[o + j] - (s + 1 < N ? d[o + np + j] : 0.0)); });
  st<TS, double>(out, o + i, sgn * (r[o + i] + v));
}

// largest |kappa(x) - kappa(x_0)| over the nodes (a constant field gives 0)
#ifndef STP_SOLVER_TU   // used by the base translation unit only
__global__ void __launch_bounds__(kBlock) k_field_spread(long nnodes, const double* __restrict__ f,
                                                         double* __restrict__ partial) {
  const double f0 = f[0];
  double m = 0.0;
  for (long q = long(blockIdx.x) * kBlock + threadIdx.x; q < nnodes; q += long(gridDim.x) * kBlock)
    m = fmax(m, fabs(f[q] - f0));
  __shared__ double red[kBlock];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
#endif

}  // namespace stp

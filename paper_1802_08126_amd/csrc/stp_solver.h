// The typed solver: every launch of an iteration for one storage type TS and
// compute type TC.  Included by one translation unit per precision.
#pragma once
#include "stp_internal.h"

namespace stpx {

template <typename TS, typename TC>
struct Solver : SolverBase {
  stp_ctx* c;
  explicit Solver(stp_ctx* ctx) : c(ctx) {}

  TC omegaJ() const { return c->dim == 1 ? TC(2.0 / 3.0) : (c->dim == 2 ? TC(4.0 / 5.0) : TC(6.0 / 7.0)); }

  // -------------------------------------------------------------------------
  // finite elements (single problem): operator kernels of stp_fem.h
  // -------------------------------------------------------------------------
  // damping of the finite-element l1-Jacobi sweeps
  TC fem_theta() const { return TC(1.6); }

  static FemW<TC> fem_w(const FemLevelW& f) {
    FemW<TC> w;
    for (int k = 0; k < 27; ++k) {
      w.m[k] = TC(f.m[k]);
      w.a[k] = TC(f.a[k]);
    }
    return w;
  }
  static FemW<double> fem_w64(const FemLevelW& f) {
    FemW<double> w;
    for (int k = 0; k < 27; ++k) {
      w.m[k] = f.m[k];
      w.a[k] = f.a[k];
    }
    return w;
  }

  // operator of a V-cycle family: (sigma table or null, c table, stride)
  void fem_family(int which, const TC*& sig, const TC*& cc, int& stride) {
    Problem& q = c->pr[0];
    if (which == VC_A) {
      sig = nullptr;
      cc = (const TC*)q.cA;
    } else {
      sig = (const TC*)q.sigH;
      cc = (const TC*)q.cH;
    }
    stride = kMaxRank;
  }

  template <int D>
  stp_status fem_level(int l, const TC* sig, const TC* cc, int stride, const TS* b, TS* out, bool add64) {
    Problem& q = c->pr[0];
    const int N = q.N;
    const int L = int(q.lv.size());
    const Level& lv = q.lv[l];
    const int* stf = &q.state->done;
    c->kt.level = l;
    const FemW<TC> w = fem_w(q.fw[l]);
    if (l == L - 1) {   // one node per slab (never the top level)
      KLAUNCH_NAMED("k_fem_coarsest", (k_fem_coarsest<TS, TC>), dim3(unsigned((N + kBlock - 1) / kBlock)), dim3(kBlock),
                    0, c->stream, N, w.m[fem_ctr<D>()], w.a[fem_ctr<D>()], sig, cc, stride, b, out, stf);
      LAUNCH_CHECK();
      return STP_OK;
    }
    const Level& lc = q.lv[l + 1];
    const TC om = fem_theta();
    const int ns = std::max(1, c->opt.sweeps);
    const dim3 gf = grid_pts(lv.g.npts, N), gc = grid_pts(lc.g.npts, N), bl(kBlock);
    TS* xa = (TS*)lv.fr;
    TS* xb = (TS*)lv.fr2;
    KLAUNCH_NAMED("k_fem_jac0", (k_fem_jac0<D, TS, TC>), gf, bl, 0, c->stream, lv.g.npts, N, w, sig, cc, stride, om,
                  b, xa, stf);
    LAUNCH_CHECK();
    for (int k = 1; k < ns; ++k) {   // further pre-sweeps
      KLAUNCH_NAMED("k_fem_sweep", (k_fem_sweep<D, TS, TC, EPI_STORE>), gf, bl, 0, c->stream, lv.g, N, w, sig, cc,
                    stride, om, b, (const TS*)xa, xb, (const FemBind*)q.fbind, stf);
      LAUNCH_CHECK();
      std::swap(xa, xb);
    }
    KLAUNCH_NAMED("k_fem_res", (k_fem_res<D, TS, TC>), gf, bl, 0, c->stream, lv.g, N, w, sig, cc, stride, b,
                  (const TS*)xa, xb, stf);
    LAUNCH_CHECK();
    KLAUNCH_NAMED("k_fem_restrict", (k_fem_restrict<D, TS, TC, D == 2>), gc, bl, 0, c->stream, lv.g, lc.g, N,
                  (const TS*)xb, (TS*)lc.b, stf);
    LAUNCH_CHECK();
    stp_status st = fem_level<D>(l + 1, sig, cc, stride, (const TS*)lc.b, (TS*)lc.e, false);
    if (st != STP_OK) return st;
    c->kt.level = l;
    KLAUNCH_NAMED("k_fem_prolong_add", (k_fem_prolong_add<D, TS, TC, D == 2>), gf, bl, 0, c->stream, lv.g, lc.g, N,
                  (const TS*)lc.e, xa, stf);
    LAUNCH_CHECK();
    for (int k = 1; k < ns; ++k) {   // post-sweeps but the last
      KLAUNCH_NAMED("k_fem_sweep", (k_fem_sweep<D, TS, TC, EPI_STORE>), gf, bl, 0, c->stream, lv.g, N, w, sig, cc,
                    stride, om, b, (const TS*)xa, xb, (const FemBind*)q.fbind, stf);
      LAUNCH_CHECK();
      std::swap(xa, xb);
    }
    if (add64)
      KLAUNCH_NAMED("k_fem_sweep<add64>", (k_fem_sweep<D, TS, TC, EPI_ADD64>), gf, bl, 0, c->stream, lv.g, N, w, sig,
                    cc, stride, om, b, (const TS*)xa, out, (const FemBind*)q.fbind, stf);
    else
      KLAUNCH_NAMED("k_fem_sweep", (k_fem_sweep<D, TS, TC, EPI_STORE>), gf, bl, 0, c->stream, lv.g, N, w, sig, cc,
                    stride, om, b, (const TS*)xa, out, (const FemBind*)q.fbind, stf);
    LAUNCH_CHECK();
    return STP_OK;
  }

  // one application of A-tilde^{-1} (which = VC_A: W1 -> += the binding's p
  // target) or of an H-tilde_k^{-1} family (VC_H1, VC_H2: W2 -> W1)
  stp_status fem_vcycle(int which) {
    Problem& q = c->pr[0];
    const TC *sig, *cc;
    int stride;
    fem_family(which, sig, cc, stride);
    const bool a = which == VC_A;
    const TS* in = (const TS*)(a ? q.W1 : q.W2);
    TS* out = (TS*)q.W1;
    if (c->spatial == STP_SPATIAL_EXACT) {   // 1-D: exact tridiagonal solves
      const FemLevelW& f = q.fw[0];
      c->kt.level = 0;
      const dim3 gr(unsigned((q.N + 63) / 64)), bl(64);
      if (a)
        KLAUNCH_NAMED("k_fem_tridiag<add64>", (k_fem_tridiag<TS, TC, EPI_ADD64>), gr, bl, 0, c->stream, q.n, q.N,
                      TC(f.m[1]), TC(f.m[0]), TC(f.a[1]), TC(f.a[0]), sig, cc, stride, in, out,
                      (const FemBind*)q.fbind, (TC*)q.tri, &q.state->done);
      else
        KLAUNCH_NAMED("k_fem_tridiag<store>", (k_fem_tridiag<TS, TC, EPI_STORE>), gr, bl, 0, c->stream, q.n, q.N,
                      TC(f.m[1]), TC(f.m[0]), TC(f.a[1]), TC(f.a[0]), sig, cc, stride, in, out,
                      (const FemBind*)q.fbind, (TC*)q.tri, &q.state->done);
      LAUNCH_CHECK();
      return STP_OK;
    }
    switch (c->dim) {
      case 2: return fem_level<2>(0, sig, cc, stride, in, out, a);
      default: return fem_level<3>(0, sig, cc, stride, in, out, a);
    }
  }

  template <int D>
  stp_status fem_mid_d() {
    Problem& q = c->pr[0];
    c->kt.level = 0;
    const TC cmid = TC((2.0 / q.N) * q.tau * q.abar[0]);
    KLAUNCH_NAMED("k_fem_apply", (k_fem_apply<D, TS, TC>), grid_pts(q.g0.npts, q.N), dim3(kBlock), 0, c->stream, q.g0,
                  q.N, fem_w(q.fw[0]), cmid, (const TS*)q.W1, (TS*)q.W2, &q.state->done);
    LAUNCH_CHECK();
    return STP_OK;
  }
  stp_status fem_mid() {
    switch (c->dim) {
      case 1: return fem_mid_d<1>();
      case 2: return fem_mid_d<2>();
      default: return fem_mid_d<3>();
    }
  }

  template <int D, int WHICH>
  stp_status fem_resid_d() {
    Problem& q = c->pr[0];
    c->kt.level = 0;
    KLAUNCH_NAMED(WHICH == 0 ? "k_fem_resid<a1>" : "k_fem_resid<a3>", (k_fem_resid<D, TS, WHICH>),
                  grid_pts(q.g0.npts, q.N), dim3(kBlock), 0, c->stream, q.g0, q.N, fem_w64(q.fw[0]),
                  (const double*)q.taus64, (const double*)q.cA64, (const FemBind*)q.fbind, &q.state->done,
                  (TS*)q.W1, q.partial);
    LAUNCH_CHECK();
    return STP_OK;
  }
  template <int WHICH>
  stp_status fem_resid() {
    switch (c->dim) {
      case 1: return fem_resid_d<1, WHICH>();
      case 2: return fem_resid_d<2, WHICH>();
      default: return fem_resid_d<3, WHICH>();
    }
  }

  template <int D, int RM>
  stp_status fused_site(Site<FuseJob>& s, int level) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = level;
    if (s.epi == EPI_ADD64)
      KLAUNCH_NAMED("k_mg_fused<add64>", (k_mg_fused<D, TS, TC, RM, EPI_ADD64>), dim3(unsigned(s.blocks)),
                    dim3(unsigned(s.threads)), s.shmem, c->stream, s.dev, int(s.jobs.size()), omegaJ());
    else
      KLAUNCH_NAMED("k_mg_fused<store>", (k_mg_fused<D, TS, TC, RM, EPI_STORE>), dim3(unsigned(s.blocks)),
                    dim3(unsigned(s.threads)), s.shmem, c->stream, s.dev, int(s.jobs.size()), omegaJ());
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int D, int RM>
  stp_status vcycle_dr(VCycle& vc) {
    const int nl = int(vc.down.size());
    stp_status st;
    if (!vc.fused.empty())   // problems solved entirely by the fused kernel
      if ((st = fused_site<D, RM>(vc.fused[0], 0)) != STP_OK) return st;
    for (int l = 0; l < nl; ++l) {
      if ((st = down_site<D, RM>(vc.down[l], l)) != STP_OK) return st;
      if ((st = downp_site(vc.downp[l], l)) != STP_OK) return st;
      if ((st = fused_site<D, RM>(vc.fused[l + 1], l + 1)) != STP_OK) return st;
    }
    for (int l = nl - 1; l >= 0; --l) {
      if ((st = up_site<D, RM>(vc.up[l], l)) != STP_OK) return st;
      if ((st = upp_site(vc.upp[l], l)) != STP_OK) return st;
    }
    return STP_OK;
  }

  template <int D, int RM>
  stp_status down_site(Site<TileJob>& s, int l) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = l;
    const dim3 gr(unsigned(s.blocks)), bl(kBlock);
    const int nj = int(s.jobs.size());
    switch (s.variant()) {   // a fixed field needs no register copy of the fields: one instantiation
      case 1: KLAUNCH_NAMED("k_mg_down", (k_mg_down<D, TS, TC, 1, 1>), gr, bl, 0, c->stream, s.dev, nj, omegaJ()); break;
      case 2: KLAUNCH_NAMED("k_mg_down", (k_mg_down<D, TS, TC, RM, 2>), gr, bl, 0, c->stream, s.dev, nj, omegaJ()); break;
      default: KLAUNCH_NAMED("k_mg_down", (k_mg_down<D, TS, TC, RM, 0>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  // register-pencil down-sweeps of level l (3-D fixed-field jobs)
  stp_status downp_site(Site<TileJob>& s, int l) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = l;
    KLAUNCH_NAMED("k_mg_down_p3", (k_mg_down_p3<TS, TC, PencilTY<TC>::v>), dim3(unsigned(s.blocks)),
                  dim3(kPencilThreads), 0,
                  c->stream, s.dev, int(s.jobs.size()), omegaJ());
    LAUNCH_CHECK();
    return STP_OK;
  }

  // register-pencil up-sweeps of level l
  stp_status upp_site(Site<TileJob>& s, int l) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = l;
    const dim3 gr(unsigned(s.blocks)), bl(kPencilThreads);
    const int nj = int(s.jobs.size());
    if (s.epi == EPI_ADD64)
      KLAUNCH_NAMED("k_mg_up_p3<add64>", (k_mg_up_p3<TS, TC, PencilUpTY<TS, EPI_ADD64>::v, EPI_ADD64>), gr, bl, 0, c->stream, s.dev,
                    nj, omegaJ());
    else if (s.epi == EPI_ADDTS)
      KLAUNCH_NAMED("k_mg_up_p3<addout>", (k_mg_up_p3<TS, TC, PencilUpTY<TS, EPI_ADDTS>::v, EPI_ADDTS>), gr, bl, 0,
                    c->stream, s.dev, nj, omegaJ());
    else
      KLAUNCH_NAMED("k_mg_up_p3<store>", (k_mg_up_p3<TS, TC, PencilUpTY<TS, EPI_STORE>::v, EPI_STORE>), gr, bl, 0, c->stream,
                    s.dev, nj, omegaJ());
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int D, int RM>
  stp_status up_site(Site<TileJob>& s, int l) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = l;
    const dim3 gr(unsigned(s.blocks)), bl(kBlock);
    const int nj = int(s.jobs.size());
    const int v = s.variant();
    if (s.epi == EPI_ADD64) {
      const char* nm = "k_mg_up<add64>";
      if (v == 1) KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, 1, EPI_ADD64, 1>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
      else if (v == 2) KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, RM, EPI_ADD64, 2>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
      else KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, RM, EPI_ADD64, 0>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
    } else {
      const char* nm = "k_mg_up<store>";
      if (v == 1) KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, 1, EPI_STORE, 1>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
      else if (v == 2) KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, RM, EPI_STORE, 2>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
      else KLAUNCH_NAMED(nm, (k_mg_up<D, TS, TC, RM, EPI_STORE, 0>), gr, bl, 0, c->stream, s.dev, nj, omegaJ());
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  // one launch of the representative site of a schedule knob
  template <int D, int RM>
  stp_status knob_dr(int knob) {
    switch (knob) {
      case KN_R0: return resid_dr<D, 0, RM>();
      case KN_R1: return resid_dr<D, 1, RM>();
      case KN_MID: return apply_dr<D, RM>(c->sites.mid);
      case KN_UPA0: return up_site<D, RM>(c->sites.vc[VC_A].up[0], 0);
      case KN_FUSE: {
        VCycle& v = c->sites.vc[VC_H1];
        for (size_t l = 0; l < v.fused.size(); ++l) {
          const stp_status st = fused_site<D, RM>(v.fused[l], int(l));
          if (st != STP_OK) return st;
        }
        return STP_OK;
      }
      default:
        if (knob < KN_UP0) return down_site<D, RM>(c->sites.vc[VC_H1].down[knob - KN_DOWN0], knob - KN_DOWN0);
        return up_site<D, RM>(c->sites.vc[VC_H1].up[knob - KN_UP0], knob - KN_UP0);
    }
  }

  stp_status launch_knob(int knob) override {
    switch (c->dim * 10 + c->rm) {
      case 11: return knob_dr<1, 1>(knob);
      case 12: return knob_dr<1, 2>(knob);
      case 14: return knob_dr<1, 4>(knob);
      case 21: return knob_dr<2, 1>(knob);
      case 22: return knob_dr<2, 2>(knob);
      case 24: return knob_dr<2, 4>(knob);
      case 31: return knob_dr<3, 1>(knob);
      case 32: return knob_dr<3, 2>(knob);
      default: return knob_dr<3, 4>(knob);
    }
  }

  // transform group g: forward (mode 0) and inverse-accumulate (mode 1) launches
  stp_status launch_transform(int g) override {
    std::vector<Site<TimeJob>> one4(1, c->sites.a4[g]), one6(1, c->sites.a6[g]);
    stp_status st = transform_sites(one4, 0);
    if (st != STP_OK) return st;
    return transform_sites(one6, 1);
  }

  // nu_A (A) or nu_H (H1, H2) cycles, each on the residual the ones before
  // it leave (multigrid only; exact solves need one).  A: cycles 1..nu-1 store
  // to Xnu, then b -= L Xnu and p += Xnu, and the last cycle adds into p.
  // H: the first cycle stores the output o, b -= L o (the tiled operator),
  // each middle cycle stores to Xnu, then o += Xnu and b -= L Xnu, and the last
  // cycle adds into o.  The steps
  // read their operands from job tables, so captured graphs follow a rebinding
  // of the A target as the cycles do.
  stp_status run_vcycle(int which) override {
    if (c->disc == STP_DISC_FEM) return fem_vcycle(which);
    const int nu = which == VC_A ? c->opt.nu_A : c->opt.nu_H;
    if (nu <= 1 || !multi_cycle(c)) return run_cycle(c->sites.vc[which]);
    const int fam = which == VC_A ? 0 : 1;
    VCycle& vx = c->sites.vc[fam == 0 ? VC_AX : VC_HX];
    stp_status st;
    if (fam == 0) {
      for (int k = 1; k < nu; ++k) {
        if ((st = run_cycle(vx)) != STP_OK) return st;
        if ((st = run_apply(c->sites.nu[0])) != STP_OK) return st;   // b -= L x, p += x
      }
      return run_cycle(c->sites.vc[which]);
    }
    if ((st = run_cycle(c->sites.vc[which])) != STP_OK) return st;
    if ((st = run_apply(c->sites.nures)) != STP_OK) return st;   // b -= L o
    for (int k = 1; k + 1 < nu; ++k) {
      if ((st = run_cycle(vx)) != STP_OK) return st;
      if ((st = run_apply(c->sites.nu[1])) != STP_OK) return st;   // b -= L x, o += x
    }
    return run_cycle(c->sites.vc[VC_HA]);
  }

  stp_status run_cycle(VCycle& vc) {
    if (c->spatial == STP_SPATIAL_EXACT) {
      Site<PointJob>& s = vc.tri;
      c->kt.level = 0;
      if (s.epi == EPI_ADD64)
        KLAUNCH_NAMED("k_tridiag<add64>", (k_tridiag<TS, TC, EPI_ADD64>), dim3(unsigned(s.blocks)), dim3(64), 0,
                      c->stream, s.dev, int(s.jobs.size()));
      else
        KLAUNCH_NAMED("k_tridiag<store>", (k_tridiag<TS, TC, EPI_STORE>), dim3(unsigned(s.blocks)), dim3(64), 0,
                      c->stream, s.dev, int(s.jobs.size()));
      LAUNCH_CHECK();
      return STP_OK;
    }
    switch (c->dim * 10 + c->rm) {
      case 11: return vcycle_dr<1, 1>(vc);
      case 12: return vcycle_dr<1, 2>(vc);
      case 14: return vcycle_dr<1, 4>(vc);
      case 21: return vcycle_dr<2, 1>(vc);
      case 22: return vcycle_dr<2, 2>(vc);
      case 24: return vcycle_dr<2, 4>(vc);
      case 31: return vcycle_dr<3, 1>(vc);
      case 32: return vcycle_dr<3, 2>(vc);
      default: return vcycle_dr<3, 4>(vc);
    }
  }

  template <int D, int RM>
  stp_status apply_dr(Site<TileJob>& s) {
    if (s.jobs.empty()) return STP_OK;
    c->kt.level = 0;
    const dim3 gr(unsigned(s.blocks)), bl(MidTile<D>::threads);
    const int nj = int(s.jobs.size());
    switch (s.variant()) {
      case 1: KLAUNCH_NAMED("k_apply_tile", (k_apply_tile<D, TS, TC, 1, 1>), gr, bl, 0, c->stream, s.dev, nj); break;
      case 2: KLAUNCH_NAMED("k_apply_tile", (k_apply_tile<D, TS, TC, RM, 2>), gr, bl, 0, c->stream, s.dev, nj); break;
      default: KLAUNCH_NAMED("k_apply_tile", (k_apply_tile<D, TS, TC, RM, 0>), gr, bl, 0, c->stream, s.dev, nj);
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status run_apply(Site<TileJob>& s) {
    switch (c->dim * 10 + c->rm) {
      case 11: return apply_dr<1, 1>(s);
      case 12: return apply_dr<1, 2>(s);
      case 14: return apply_dr<1, 4>(s);
      case 21: return apply_dr<2, 1>(s);
      case 22: return apply_dr<2, 2>(s);
      case 24: return apply_dr<2, 4>(s);
      case 31: return apply_dr<3, 1>(s);
      case 32: return apply_dr<3, 2>(s);
      default: return apply_dr<3, 4>(s);
    }
  }

  stp_status run_mid() { return c->disc == STP_DISC_FEM ? fem_mid() : run_apply(c->sites.mid); }

  template <int L1, int L2, int MODE, int ACC>
  stp_status fft2_site(Site<TimeJob>& s) {
    constexpr int C = kBlock / (1 << L1);
    const size_t lds = size_t(1 << (L1 + L2)) * C * sizeof(TC);
    KLAUNCH_NAMED(MODE == MODE_A4 ? "k_time_fft2<a4>" : (ACC ? "k_time_fft2<a6,add64>" : "k_time_fft2<a6>"),
                  (k_time_fft2<TS, TC, MODE, ACC, L1, L2>), dim3(unsigned(s.blocks)), dim3(kBlock), lds, c->stream,
                  s.dev, int(s.jobs.size()));
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int MODE, int ACC>
  stp_status fft2_dispatch(Site<TimeJob>& s) {
    switch (s.key) {
      case 4: return fft2_site<1, 1, MODE, ACC>(s);
      case 8: return fft2_site<2, 1, MODE, ACC>(s);
      case 16: return fft2_site<2, 2, MODE, ACC>(s);
      case 32: return fft2_site<3, 2, MODE, ACC>(s);
      case 64: return fft2_site<3, 3, MODE, ACC>(s);
      case 128: return fft2_site<4, 3, MODE, ACC>(s);
      default: return fft2_site<4, 4, MODE, ACC>(s);
    }
  }

  // timing records of transform site g carry "level" g
  stp_status transform_sites(std::vector<Site<TimeJob>>& sites, int mode) {
    for (size_t g = 0; g < sites.size(); ++g) {
      Site<TimeJob>& s = sites[g];
      c->kt.level = int(g);
      if (s.jobs.empty()) continue;
      const bool acc = s.epi != 0;
      if (s.path == TP_DENSE) {
        if (acc)
          KLAUNCH_NAMED("k_time_dense<a6,add64>", (k_time_dense<TS, TC, 1>), dim3(unsigned(s.blocks)), dim3(kBlock), 0,
                        c->stream, s.dev, int(s.jobs.size()));
        else
          KLAUNCH_NAMED(mode == 0 ? "k_time_dense<a4>" : "k_time_dense<a6>", (k_time_dense<TS, TC, 0>),
                        dim3(unsigned(s.blocks)), dim3(kBlock), 0, c->stream, s.dev, int(s.jobs.size()));
        LAUNCH_CHECK();
        continue;
      }
      if (s.path == TP_FFT2) {
        stp_status st;
        if (mode == 0) st = fft2_dispatch<MODE_A4, 0>(s);
        else if (acc) st = fft2_dispatch<MODE_A6, 1>(s);
        else st = fft2_dispatch<MODE_A6, 0>(s);
        if (st != STP_OK) return st;
        continue;
      }
      const int C = s.C;
      const size_t lds = s.lds;
      if (s.path == TP_BLUESTEIN) {   // every job of the site has the same M
        if (mode == 0)
          KLAUNCH_NAMED("k_time_bluestein<a4>", (k_time_bluestein<TS, TC, MODE_A4, 0>), dim3(unsigned(s.blocks)),
                        dim3(kBlock), lds, c->stream, s.dev, int(s.jobs.size()), C);
        else if (acc)
          KLAUNCH_NAMED("k_time_bluestein<a6,add64>", (k_time_bluestein<TS, TC, MODE_A6, 1>), dim3(unsigned(s.blocks)),
                        dim3(kBlock), lds, c->stream, s.dev, int(s.jobs.size()), C);
        else
          KLAUNCH_NAMED("k_time_bluestein<a6>", (k_time_bluestein<TS, TC, MODE_A6, 0>), dim3(unsigned(s.blocks)),
                        dim3(kBlock), lds, c->stream, s.dev, int(s.jobs.size()), C);
        LAUNCH_CHECK();
        continue;
      }
      if (s.path == TP_FOUR) {   // two passes over the scratch
        const dim3 gr(unsigned(s.blocks)), bl(kBlock);
        const int nj = int(s.jobs.size());
        if (mode == 0) {
          KLAUNCH_NAMED("k_time_fft4<a4,p0>", (k_time_fft4<TS, TC, MODE_A4, 0, 0>), gr, bl, lds, c->stream, s.dev, nj, C);
          LAUNCH_CHECK();
          KLAUNCH_NAMED("k_time_fft4<a4,p1>", (k_time_fft4<TS, TC, MODE_A4, 1, 0>), gr, bl, lds, c->stream, s.dev, nj, C);
        } else {
          KLAUNCH_NAMED("k_time_fft4<a6,p0>", (k_time_fft4<TS, TC, MODE_A6, 0, 0>), gr, bl, lds, c->stream, s.dev, nj, C);
          LAUNCH_CHECK();
          if (acc)
            KLAUNCH_NAMED("k_time_fft4<a6,p1,add64>", (k_time_fft4<TS, TC, MODE_A6, 1, 1>), gr, bl, lds, c->stream,
                          s.dev, nj, C);
          else
            KLAUNCH_NAMED("k_time_fft4<a6,p1>", (k_time_fft4<TS, TC, MODE_A6, 1, 0>), gr, bl, lds, c->stream, s.dev,
                          nj, C);
        }
        LAUNCH_CHECK();
        continue;
      }
      // Stockham: every job of the site has the same N, hence the same layout
      if (mode == 0)
        KLAUNCH_NAMED("k_time_fft<a4>", (k_time_fft<TS, TC, MODE_A4, 0>), dim3(unsigned(s.blocks)), dim3(kBlock), lds,
                      c->stream, s.dev, int(s.jobs.size()), C);
      else if (acc)
        KLAUNCH_NAMED("k_time_fft<a6,add64>", (k_time_fft<TS, TC, MODE_A6, 1>), dim3(unsigned(s.blocks)), dim3(kBlock),
                      lds, c->stream, s.dev, int(s.jobs.size()), C);
      else
        KLAUNCH_NAMED("k_time_fft<a6>", (k_time_fft<TS, TC, MODE_A6, 0>), dim3(unsigned(s.blocks)), dim3(kBlock), lds,
                      c->stream, s.dev, int(s.jobs.size()), C);
      LAUNCH_CHECK();
    }
    return STP_OK;
  }

  // H-tilde^{-1}: W1 holds r on entry; Phi^{-1} yhat goes to the a6 targets.
  stp_status run_precH() override {
    stp_status s;
    c->kt.phase = PH_DST;
    if ((s = transform_sites(c->sites.a4, 0)) != STP_OK) return s;   // rhat = Phi^{-T} r    (W1 -> W2)
    c->kt.phase = PH_HBLOCK;
    if ((s = run_vcycle(VC_H1)) != STP_OK) return s;                  // x = H~_k^{-1} rhat   (W2 -> W1)
    if ((s = run_mid()) != STP_OK) return s;                          // y = (2/N) tau A x    (W1 -> W2)
    if ((s = run_vcycle(VC_H2)) != STP_OK) return s;                  // yhat = H~_k^{-1} y   (W2 -> W1)
    c->kt.phase = PH_DST;
    s = transform_sites(c->sites.a6, 1);                              // += alpha Phi^{-1} yhat
    c->kt.phase = PH_OTHER;
    return s;
  }

  template <int D, int WHICH, int RM>
  stp_status resid_dr() {
    Site<ResidJob>& s = c->sites.resid[WHICH];
    c->kt.level = 0;
    const char* nm = WHICH == 0 ? "k_resid_tile<a1>" : "k_resid_tile<a3>";
    const dim3 gr(unsigned(s.blocks)), bl(ResidTile<D>::threads);
    const int nj = int(s.jobs.size());
    switch (s.variant()) {
      case 1: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, 1, 1>), gr, bl, 0, c->stream, s.dev, nj); break;
      case 2: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, RM, 2>), gr, bl, 0, c->stream, s.dev, nj); break;
      default: KLAUNCH_NAMED(nm, (k_resid_tile<D, TS, WHICH, RM, 0>), gr, bl, 0, c->stream, s.dev, nj);
    }
    LAUNCH_CHECK();
    return STP_OK;
  }

  template <int WHICH>
  stp_status run_resid() {
    switch (c->dim * 10 + c->rm) {
      case 11: return resid_dr<1, WHICH, 1>();
      case 12: return resid_dr<1, WHICH, 2>();
      case 14: return resid_dr<1, WHICH, 4>();
      case 21: return resid_dr<2, WHICH, 1>();
      case 22: return resid_dr<2, WHICH, 2>();
      case 24: return resid_dr<2, WHICH, 4>();
      case 31: return resid_dr<3, WHICH, 1>();
      case 32: return resid_dr<3, WHICH, 2>();
      default: return resid_dr<3, WHICH, 4>();
    }
  }

  stp_status iteration(bool full = true) override {
    stp_status s;
    const bool fem = c->disc == STP_DISC_FEM;
    c->kt.phase = PH_RESID;
    if ((s = fem ? fem_resid<0>() : run_resid<0>()) != STP_OK) return s;   // r_p = K u - A p - f   -> W1
    c->kt.phase = PH_ATILDE;
    if ((s = run_vcycle(VC_A)) != STP_OK) return s;      // p += A~^{-1} r_p
    c->kt.phase = PH_RESID;
    if ((s = fem ? fem_resid<1>() : run_resid<1>()) != STP_OK) return s;   // r_u -> W1, partials of ||f - B u||^2
    if ((s = launch_finalize(c)) != STP_OK) return s;   // stop test and divergence guard
    c->kt.phase = PH_OTHER;
    return full ? run_precH() : STP_OK;                  // u += omega H~^{-1} r_u
  }

  stp_status cast_out(const void* a, double scale, double* b, long n) override {
    KLAUNCH((k_cast_scale64<TS>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n,
            (const TS*)a, scale, b);
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status resid(int which) override {
    if (c->disc == STP_DISC_FEM) return which == 0 ? fem_resid<0>() : fem_resid<1>();
    return which == 0 ? run_resid<0>() : run_resid<1>();
  }

  stp_status kt_add_in(const double* r, const double* d, double sgn) override {
    Problem& q = c->pr[0];
    const long nv = long(q.N) * q.g0.npts;
    if (c->disc == STP_DISC_FEM) {
      const FemW<double> w = fem_w64(q.fw[0]);
      const dim3 gr = grid_pts(q.g0.npts, q.N);
      switch (c->dim) {
        case 1: KLAUNCH((k_fem_kt_add_cast<1, TS>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, r, d, sgn, (TS*)q.W1); break;
        case 2: KLAUNCH((k_fem_kt_add_cast<2, TS>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, r, d, sgn, (TS*)q.W1); break;
        default: KLAUNCH((k_fem_kt_add_cast<3, TS>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, r, d, sgn, (TS*)q.W1);
      }
      LAUNCH_CHECK();
      return STP_OK;
    }
    KLAUNCH((k_kt_add_cast<TS>), dim3(unsigned((nv + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
            q.g0.npts, q.N, r, d, sgn, (TS*)q.W1);
    LAUNCH_CHECK();
    return STP_OK;
  }

  stp_status cast_in(const double* a, void* b, long n) override {
    KLAUNCH((k_cast_from64<TS>), dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n, a, (TS*)b);
    LAUNCH_CHECK();
    return STP_OK;
  }

  // the Stockham kernels may take up to the whole LDS of a CU
  stp_status init() override {
    {   // the 16-point twiddles of this translation unit's transform kernels
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
    const int lds = 160 * 1024;
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A4, 0>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A6, 0>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_fft<TS, TC, MODE_A6, 1>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_bluestein<TS, TC, MODE_A4, 0>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_bluestein<TS, TC, MODE_A6, 0>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    HIP_TRY(hipFuncSetAttribute((const void*)k_time_bluestein<TS, TC, MODE_A6, 1>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    for (const void* f : {(const void*)k_time_fft4<TS, TC, MODE_A4, 0, 0>, (const void*)k_time_fft4<TS, TC, MODE_A4, 1, 0>,
                          (const void*)k_time_fft4<TS, TC, MODE_A6, 0, 0>, (const void*)k_time_fft4<TS, TC, MODE_A6, 1, 0>,
                          (const void*)k_time_fft4<TS, TC, MODE_A6, 1, 1>})
      HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    return STP_OK;
  }

  stp_status setup_problem(Problem& q) override {
    const int N = q.N, R = q.R;
    std::vector<TC> cA(size_t(N) * kMaxRank, TC(0)), cH(size_t(N) * kMaxRank, TC(0)), sig(N), mid(kMaxRank, TC(0));
    std::vector<double> cA64(size_t(N) * kMaxRank, 0.0);
    for (int s = 0; s < N; ++s)
      for (int r = 0; r < R; ++r) {
        cA64[size_t(s) * kMaxRank + r] = q.taus[s] * q.tcoef[size_t(r) * N + s];
        cA[size_t(s) * kMaxRank + r] = TC(q.taus[s] * q.tcoef[size_t(r) * N + s]);
        cH[size_t(s) * kMaxRank + r] = TC(q.tau * q.abar[r]);
      }
    for (int k = 0; k < N; ++k) sig[k] = TC(2.0 * std::sin((2.0 * k + 1.0) * M_PI / (4.0 * N)));
    for (int r = 0; r < R; ++r) mid[r] = TC((2.0 / N) * q.tau * q.abar[r]);
    HIP_TRY(hipMemcpyAsync(q.cA64, cA64.data(), cA64.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(q.taus64, q.taus.data(), size_t(N) * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(q.cA, cA.data(), cA.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(q.cH, cH.data(), cH.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(q.sigH, sig.data(), sig.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(q.cMid, mid.data(), mid.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
    if (q.sinT) {
      std::vector<TC> sT(size_t(N) * N), sM(size_t(N) * N);
      for (int k = 0; k < N; ++k)
        for (int m = 0; m < N; ++m) {
          // sin((2k+1)(m+1) pi / (2N)) with the angle reduced exactly in integers
          const long qq = (long(2 * k + 1) * long(m + 1)) % (4L * N);
          const double v = std::sin(double(qq) * M_PI / (2.0 * N));
          sT[size_t(k) * N + m] = TC(v);
          sM[size_t(m) * N + k] = TC(v);
        }
      HIP_TRY(hipMemcpyAsync(q.sinT, sT.data(), sT.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(q.sinM, sM.data(), sM.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    }
    if (q.blM) {
      // Bluestein tables: w_M^m, w_{4N}^m, chirp c_n = exp(-i pi (n^2 mod 2N) / N),
      // and Bhat = DFT_M(b) / M with b_m = b_{M-m} = conj(c_m) (|m| < N), by
      // direct sums with exactly reduced angles
      const int M = q.blM;
      std::vector<TC> twm(2 * size_t(M)), tw4(2 * size_t(N)), ch(2 * size_t(N)), bh(2 * size_t(M));
      std::vector<double> cr(N), ci(N);
      for (int m = 0; m < M; ++m) {
        twm[m] = TC(std::cos(2.0 * M_PI * m / M));
        twm[M + m] = TC(-std::sin(2.0 * M_PI * m / M));
      }
      for (int m = 0; m < N; ++m) {
        tw4[m] = TC(std::cos(M_PI * m / (2.0 * N)));
        tw4[N + m] = TC(-std::sin(M_PI * m / (2.0 * N)));
        const long sq = (long(m) * long(m)) % (2L * N);
        cr[m] = std::cos(M_PI * double(sq) / N);
        ci[m] = -std::sin(M_PI * double(sq) / N);
        ch[m] = TC(cr[m]);
        ch[N + m] = TC(ci[m]);
      }
      for (int k = 0; k < M; ++k) {
        double sr = cr[0], si = -ci[0];   // m = 0
        for (int m = 1; m < N; ++m) {
          // b_m = b_{M-m} = conj(c_m): b_m w^{mk} + b_m w^{-mk} = 2 conj(c_m) cos(2 pi m k / M)
          const long r = (long(m) * long(k)) % M;
          const double cs = std::cos(2.0 * M_PI * double(r) / M);
          sr += 2.0 * cr[m] * cs;
          si -= 2.0 * ci[m] * cs;
        }
        bh[k] = TC(sr / M);
        bh[M + k] = TC(si / M);
      }
      HIP_TRY(hipMemcpyAsync(q.tw, twm.data(), twm.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(q.tw4, tw4.data(), tw4.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(q.chirp, ch.data(), ch.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(q.bhat, bh.data(), bh.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    } else if (q.tw) {
      std::vector<TC> tw(2 * size_t(N)), tw4(2 * size_t(N));
      for (int m = 0; m < N; ++m) {
        tw[m] = TC(std::cos(2.0 * M_PI * m / N));
        tw[N + m] = TC(-std::sin(2.0 * M_PI * m / N));
        tw4[m] = TC(std::cos(M_PI * m / (2.0 * N)));
        tw4[N + m] = TC(-std::sin(M_PI * m / (2.0 * N)));
      }
      HIP_TRY(hipMemcpyAsync(q.tw, tw.data(), tw.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(q.tw4, tw4.data(), tw4.size() * sizeof(TC), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    }
    // level fields: restrict unscaled float64 fields, then scale by 0.5/h^2 into TC
    for (size_t l = 0; l < q.lv.size(); ++l) {
      Level& L = q.lv[l];
      const long nn = L.g.nnodes;
      if (l > 0) {
        Level& Fl = q.lv[l - 1];
        for (int r = 0; r < R; ++r) {
          const dim3 gr(unsigned((nn + kBlock - 1) / kBlock));
          switch (q.dim) {
            case 1: KLAUNCH(k_restrict_kappa<1>, gr, dim3(kBlock), 0, c->stream, Fl.n, L.n, Fl.kraw + r * Fl.g.nnodes, L.kraw + r * nn); break;
            case 2: KLAUNCH(k_restrict_kappa<2>, gr, dim3(kBlock), 0, c->stream, Fl.n, L.n, Fl.kraw + r * Fl.g.nnodes, L.kraw + r * nn); break;
            default: KLAUNCH(k_restrict_kappa<3>, gr, dim3(kBlock), 0, c->stream, Fl.n, L.n, Fl.kraw + r * Fl.g.nnodes, L.kraw + r * nn); break;
          }
          LAUNCH_CHECK();
        }
      }
      const double sc = 0.5 / (L.h * L.h);
      const long tot = nn * R;
      KLAUNCH((k_scale_copy<TC>), dim3(unsigned((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, tot,
              (const double*)L.kraw, sc, (TC*)L.kscaled);
      LAUNCH_CHECK();
      if (l == 0) {
        KLAUNCH((k_scale_copy<double>), dim3(unsigned((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
                tot, (const double*)L.kraw, sc, q.kap64);
        LAUNCH_CHECK();
      }
    }
    // fixed fields and face sums of the register-pencil down-sweeps
    for (size_t l = 0; l < q.lv.size(); ++l)
      for (int fam = 0; fam < 2; ++fam) {
        Level& L = q.lv[l];
        if (!L.pen[fam]) continue;
        const long nb = std::min(4096L, (L.g.npts + kBlock - 1) / kBlock);
        KLAUNCH((k_pencil_fields<TC>), dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, L.g,
                family_op(q, int(l), fam), (TC*)L.pk[fam], (TC*)L.pd[fam]);
        LAUNCH_CHECK();
      }
    return STP_OK;
  }
};

}  // namespace stpx

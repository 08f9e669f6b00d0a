// Host side of the space-time Uzawa solver: problem setup, multigrid
// hierarchy, workspace planning, merged (batched) launch tables, the
// iteration driver with HIP-graph replay, and the C ABI of stp.h.
//
// A context holds a batch of P >= 1 independent problems of one spatial
// dimension.  Every step of an Uzawa iteration is one merged launch per
// kernel instantiation ("site") that serves all problems at once; a site is a
// table of jobs, one per problem, that the kernels search by block index.
#include "stp_internal.h"

#include <atomic>
#include <chrono>
#include <cstdarg>

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
// device bytes obtained with hipMalloc by the library in this process (diagnostic)
static std::atomic<size_t> g_dev_bytes{0};

namespace stpx {
stp_status fail(stp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}
}  // namespace stpx

namespace stpx {
stp_status launch_finalize(stp_ctx* c) {
  c->kt.level = 0;
  // one block per job of the table: the problems the tables cover (a batch
  // solve drops stopped problems from them)
  const size_t nf = c->sites.fin.size();
  if (nf == 0) return STP_OK;
  KLAUNCH(k_finalize, dim3(unsigned(nf)), dim3(kBlock), 0, c->stream, (const FinJob*)c->sites.fin_dev);
  LAUNCH_CHECK();
  return STP_OK;
}
}  // namespace stpx

namespace {

constexpr int kDotBlocks = 512;   // partial sums of the setup dot products

// Doubles of setup and tuning scratch a context needs: the omega estimate
// (five float64 vectors per problem and the dot partials, only when omega is
// estimated), the autotuner (two float64 vectors per problem) and the kappa
// check (block partials of one problem's node count); the three uses never
// overlap in time, so they share one region.
size_t scratch_doubles(const stp_ctx* c) {
  size_t est = 0, tune = 0, kap = 0;
  for (const Problem& q : c->pr) {
    const size_t nv = size_t(q.N) * size_t(q.g0.npts);
    est += 5 * nv;
    tune += 2 * nv;
    kap = std::max(kap, size_t((q.g0.nnodes + kBlock - 1) / kBlock) + kMaxRank);
  }
  if (c->opt.omega > 0 || c->spatial == STP_SPATIAL_NONE) est = 0;
  else est += c->pr.size() * (kDotBlocks + 1);
  return std::max(est, std::max(tune, kap));
}

// Scratch for one use: the region of the caller's workspace, or (when the
// library owns the workspace) an allocation held until scratch_put.
stp_status scratch_get(stp_ctx* c, size_t n, double** out, bool* owned) {
  *owned = false;
  if (c->scratch_n) {
    if (n > c->scratch_n) return fail(STP_EDEVICE, "scratch of %zu doubles exceeds its reservation", n);
    *out = c->scratch;
    return STP_OK;
  }
  if (hipMalloc((void**)out, std::max<size_t>(n, 1) * 8) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(STP_ENOMEM, "hipMalloc of %zu bytes of scratch failed", n * 8);
  }
  g_dev_bytes += std::max<size_t>(n, 1) * 8;
  *owned = true;
  return STP_OK;
}

void scratch_put(stp_ctx* c, double* p, bool owned) {
  (void)hipStreamSynchronize(c->stream);
  if (owned && p) (void)hipFree(p);
}

// slabs per block for a launch over `tiles` tiles and S slabs: enough blocks
// to fill the chip several times over, otherwise runs of up to 16 slabs
int pick_sb(long tiles, int S) {
  long sb = (tiles * S) / 2048;
  return int(std::max(1L, std::min(16L, sb)));
}

// heuristic slabs per block scaled by 2^e, within [1, min(16, S)]
int sched_sb(long tiles, int S, int e) {
  long sb = pick_sb(tiles, S);
  sb = e >= 0 ? (sb << e) : (sb >> (-e));
  return int(std::max(1L, std::min(long(std::min(16, S)), sb)));
}

long tiles_down_d(int dim, int nc) {
  return dim == 1 ? tiles_for<1, DownTile<1>>(nc) : dim == 2 ? tiles_for<2, DownTile<2>>(nc)
                                                             : tiles_for<3, DownTile<3>>(nc);
}
long tiles_up_d(int dim, int n) {
  return dim == 1 ? tiles_for<1, UpTile<1>>(n) : dim == 2 ? tiles_for<2, UpTile<2>>(n) : tiles_for<3, UpTile<3>>(n);
}
long tiles_mid_d(int dim, int n) {
  return dim == 1 ? tiles_for<1, MidTile<1>>(n) : dim == 2 ? tiles_for<2, MidTile<2>>(n) : tiles_for<3, MidTile<3>>(n);
}
long tiles_resid_d(int dim, int n) {
  return dim == 1 ? tiles_for<1, ResidTile<1>>(n) : dim == 2 ? tiles_for<2, ResidTile<2>>(n)
                                                             : tiles_for<3, ResidTile<3>>(n);
}


// Plan (dry run) or carve (real run) one problem's buffers.
void plan_problem(int prec, int spatial, Problem& q, Bump& bp, bool nux, bool fem) {
  const size_t tsb = ts_bytes(prec), tcb = tc_bytes(prec);
  const long N = q.N;
  {
    int C;
    size_t lds;
    transform_path(q.N, tcb, q.tpath, C, lds);
  }
  q.resid_tiles = tiles_resid_d(q.dim, q.n);
  const dim3 gp = grid_pts(q.g0.npts, q.N);
  q.nfnorm = long(gp.x) * gp.y * gp.z;
  q.state = (DevState*)bp.take(sizeof(DevState));
  // residual partials for any slabs-per-block choice (at most one slab per block)
  q.partial = (double*)bp.take(size_t(std::max(q.resid_tiles * q.N, q.nfnorm)) * 8);
  // norm partials of a returned pair: one row each for r_p and r_u (FEM: one per
  // block of its grid; else one per block of the up-sweep tiles' default schedule)
  q.nrm = (double*)bp.take(size_t(2) * std::max(long(kNormBlocks), tiles_up_d(q.dim, q.n) * N) * 8);
  q.njob = bp.take(sizeof(ResidJob));
  q.fbind = fem ? (FemBind*)bp.take(sizeof(FemBind)) : nullptr;
  q.kap64 = (double*)bp.take(size_t(q.R) * q.g0.nnodes * 8);
  q.cA64 = (double*)bp.take(size_t(N) * kMaxRank * 8);
  q.taus64 = (double*)bp.take(size_t(N) * 8);
  q.cA = bp.take(size_t(N) * kMaxRank * tcb);
  q.cH = bp.take(size_t(N) * kMaxRank * tcb);
  q.sigH = bp.take(size_t(N) * tcb);
  q.cMid = bp.take(size_t(kMaxRank) * tcb);
  q.tw = q.tw4 = q.sinT = q.sinM = nullptr;
  // tables of every path the step count can take: dense (default path, or
  // a candidate for N <= 64) and the FFT twiddles (powers of two <= 4096)
  q.chirp = q.bhat = nullptr;
  q.blM = 0;
  if (q.tpath == TP_DENSE || q.N <= 64) {
    q.sinT = bp.take(size_t(N) * N * tcb);
    q.sinM = bp.take(size_t(N) * N * tcb);
  }
  q.fs = nullptr;
  if (is_pow2(q.N) && q.N <= kFourMaxN) {
    q.tw = bp.take(size_t(2) * N * tcb);
    q.tw4 = bp.take(size_t(2) * N * tcb);
    if (four_step_n(q.N, tcb)) q.fs = bp.take(size_t(2) * N * q.g0.npts * tcb);   // four-step scratch
  } else if (q.N <= kBlueMaxN) {
    q.blM = bluestein_M(q.N);
    q.tw = bp.take(size_t(2) * q.blM * tcb);
    q.tw4 = bp.take(size_t(2) * N * tcb);
    q.chirp = bp.take(size_t(2) * N * tcb);
    q.bhat = bp.take(size_t(2) * q.blM * tcb);
  }
  q.W1 = bp.take(size_t(N) * q.g0.npts * tsb);
  q.W2 = bp.take(size_t(N) * q.g0.npts * tsb);
  q.Xnu = nux ? bp.take(size_t(N) * q.g0.npts * tsb) : nullptr;
  q.tri = (spatial == STP_SPATIAL_EXACT) ? bp.take(size_t(2) * N * q.n * tcb) : nullptr;
  for (size_t l = 0; l < q.lv.size(); ++l) {
    Level& L = q.lv[l];
    L.kraw = (l == 0) ? const_cast<double*>(q.fields) : (double*)bp.take(size_t(q.R) * L.g.nnodes * 8);
    L.kscaled = bp.take(size_t(q.R) * L.g.nnodes * tcb);
    const size_t vb = size_t(N) * L.g.npts * tsb;
    L.b = (l == 0) ? nullptr : bp.take(vb);
    L.e = (l == 0) ? nullptr : bp.take(vb);
    const bool fx = fem && spatial == STP_SPATIAL_MG && l + 1 < q.lv.size();
    L.fr = fx ? bp.take(vb) : nullptr;
    L.fr2 = fx ? bp.take(vb) : nullptr;
    for (int fam = 0; fam < 2; ++fam) {
      const bool pen = int(l) < q.fuse_top &&
                       pencil_level(q.dim, spatial, fem, q.R, L.n, q.lv[l + 1].n, tsb, tcb, fam);
      L.pen[fam] = pen;
      L.pk[fam] = pen ? bp.take(size_t(L.g.npts) * tcb) : nullptr;
      L.pd[fam] = pen ? bp.take(size_t(L.g.npts) * tcb) : nullptr;
    }
  }
}

// Finite-element stencils of M and A (coefficient kap0) on a uniform mesh with
// n interior nodes per axis, times scale: P1 in 1-D and 2-D (squares split by
// the lower-left/upper-right diagonal), Q1 in 3-D; index ((dz+1)*3 + (dy+1))*3
// + (dx+1).  Element integrals: 1-D mass (h/6)(1, 4, 1), stiffness (1/h)(-1, 2,
// -1); 2-D P1 mass (h^2/12)(6 at the node, 1 at the four edge neighbours and the
// two diagonal neighbours along the split), stiffness (4, -1 x 4); 3-D Q1
// tensor products of the 1-D mass and stiffness.
FemLevelW fem_stencils(int dim, int n, double kap0, double scale) {
  FemLevelW w{};
  const double h = 1.0 / (n + 1);
  auto m1 = [&](int o) { return (h / 6.0) * (o == 0 ? 4.0 : 1.0); };
  auto k1 = [&](int o) { return (o == 0 ? 2.0 : -1.0) / h; };
  if (dim == 1) {
    for (int dx = -1; dx <= 1; ++dx) {
      w.m[dx + 1] = m1(dx);
      w.a[dx + 1] = kap0 * k1(dx);
    }
  } else if (dim == 2) {
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int k = (dy + 1) * 3 + (dx + 1);
        const bool ctr = dx == 0 && dy == 0, edge = (dx == 0) != (dy == 0), diag = dx != 0 && dx == dy;
        w.m[k] = (h * h / 12.0) * (ctr ? 6.0 : (edge || diag) ? 1.0 : 0.0);
        w.a[k] = kap0 * (ctr ? 4.0 : edge ? -1.0 : 0.0);
      }
  } else {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int k = ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1);
          w.m[k] = m1(dx) * m1(dy) * m1(dz);
          w.a[k] = kap0 * (k1(dx) * m1(dy) * m1(dz) + m1(dx) * k1(dy) * m1(dz) + m1(dx) * m1(dy) * k1(dz));
        }
  }
  for (int k = 0; k < 27; ++k) {
    w.m[k] *= scale;
    w.a[k] *= scale;
  }
  return w;
}

FemW<double> fem_w64(const Problem& q) {
  FemW<double> w;
  for (int k = 0; k < 27; ++k) {
    w.m[k] = q.fw[0].m[k];
    w.a[k] = q.fw[0].a[k];
  }
  return w;
}

// largest level (interior nodes per axis) of the fused coarse kernel: four
// node arrays per level stay within 64 KB of LDS in float64
int fuse_side(int dim) { return dim == 1 ? 255 : (dim == 2 ? 31 : 7); }

int fuse_threads(int e) { return 256 << std::max(0, std::min(2, e)); }

size_t fuse_lds(int dim, const FuseJob& j, size_t tcb) {
  size_t t = 0;
  for (int l = 0; l < j.nlev; ++l) {
    const size_t m = size_t(j.n[l]) + 2;
    t += 4 * (dim == 1 ? m : (dim == 2 ? m * m : m * m * m)) * tcb;
  }
  return t;
}

stp_status build_levels(int spatial, Problem& q) {
  q.lv.clear();
  int n = q.n;
  while (true) {
    Level L{};
    L.n = n;
    L.h = 1.0 / (n + 1);
    L.g.n = n;
    L.g.npts = ipow(n, q.dim);
    L.g.nnodes = ipow(n + 2, q.dim);
    q.lv.push_back(L);
    if (spatial == STP_SPATIAL_EXACT || spatial == STP_SPATIAL_NONE || n == 1) break;
    if (n % 2 == 0) return fail(STP_EUNSUPPORTED, "multigrid needs n = 2^L - 1 interior nodes per axis (got %d)", q.n);
    n = (n - 1) / 2;
    if (int(q.lv.size()) >= STP_MAX_LEVELS) return fail(STP_EUNSUPPORTED, "too many multigrid levels");
  }
  q.g0 = q.lv[0].g;
  // levels with at most fuse_side(dim) nodes per axis run inside one fused kernel
  q.fuse_top = int(q.lv.size()) - 1;
  while (q.fuse_top > 0 && q.lv[q.fuse_top - 1].n <= fuse_side(q.dim)) --q.fuse_top;
  return STP_OK;
}

// ---------------------------------------------------------------------------
// sites of the iteration (merged launches over the batch)
// ---------------------------------------------------------------------------
// problem i is in the launch tables (all of them unless a solve compacted them)
inline bool act(const stp_ctx* c, size_t i) { return c->active.empty() || c->active[i]; }

// top-level input / output of a V-cycle instance for one problem
struct VTop {
  const void* in;
  void* out;       // TS output (or null)
  double* acc64;   // float64 accumulation target (or null)
};

// acc: the finest up-sweep adds into the float64 targets (else stores);
// addout: the stored result is added into the output instead
void build_vcycle(stp_ctx* c, VCycle& vc, int fam, const std::vector<VTop>& top, bool acc, bool addout = false) {
  int Lmax = 0;
  for (auto& q : c->pr) Lmax = std::max(Lmax, int(q.lv.size()));
  vc.down.assign(std::max(0, Lmax - 1), Site<TileJob>());
  vc.downp.assign(std::max(0, Lmax - 1), Site<TileJob>());
  vc.upp.assign(std::max(0, Lmax - 1), Site<TileJob>());
  vc.up.assign(std::max(0, Lmax - 1), Site<TileJob>());
  vc.fused.assign(Lmax, Site<FuseJob>());
  vc.tri = Site<PointJob>();
  const int pty = c->prec == STP_PREC_F64 ? PencilTY<double>::v : PencilTY<float>::v;
  for (size_t i = 0; i < c->pr.size(); ++i) {
    if (!act(c, i)) continue;
    Problem& q = c->pr[i];
    const VTop& T = top[i];
    if (c->spatial == STP_SPATIAL_EXACT) {
      PointJob j{};
      j.total = q.N;
      j.g = q.lv[0].g;
      j.op = family_op(q, 0, fam);
      j.b = T.in;
      j.out = T.out;
      j.acc64 = T.acc64;
      j.scratch = q.tri;
      j.state = &q.state->done;
      vc.tri.add(j, (q.N + 63) / 64);
      vc.tri.epi = acc ? EPI_ADD64 : EPI_STORE;
      continue;
    }
    if (c->spatial != STP_SPATIAL_MG) continue;   // operators only: no V-cycle launches
    const int Lq = int(q.lv.size());
    const int ft = q.fuse_top;
    for (int l = 0; l < ft; ++l) {
      TileJob d{};
      d.gf = q.lv[l].g;
      d.gc = q.lv[l + 1].g;
      d.op = family_op(q, l, fam);
      d.b = (l == 0) ? T.in : q.lv[l].b;
      d.out = q.lv[l + 1].b;
      d.state = &q.state->done;
      if (q.lv[l].pen[fam]) {   // register pencils: a launch of their own, so a job's arithmetic
        d.tiles = int(pencil_tiles(q.lv[l + 1].n, pty));   // never depends on its batch
        d.sb = kPencilSlabs;
        d.pk = q.lv[l].pk[fam];
        d.pd = q.lv[l].pd[fam];
        vc.downp[l].add(d, long(d.tiles) * ((q.N + d.sb - 1) / d.sb), true);
      } else {
        d.tiles = int(tiles_down_d(q.dim, q.lv[l + 1].n));
        d.sb = sched_sb(d.tiles, q.N, c->sched.e[KN_DOWN0 + l]);
        vc.down[l].add(d, long(d.tiles) * ((q.N + d.sb - 1) / d.sb), d.op.cmode != CM_SLAB);
      }
      TileJob u{};
      u.gf = q.lv[l].g;
      u.gc = q.lv[l + 1].g;
      u.op = d.op;
      u.b = d.b;
      u.e = q.lv[l + 1].e;
      u.out = (l == 0) ? T.out : q.lv[l].e;
      u.acc64 = (l == 0) ? T.acc64 : nullptr;
      u.addout = (l == 0 && addout) ? 1 : 0;
      u.state = d.state;
      // float32 and bfloat16: the float64 up-sweep pencil measured slower than the
      // tiles (two rows, 270 VGPRs: 11.1 vs 10.4 ms storing on 255^3 x 64; one row:
      // faster at level 0, slower at level 1)
      const bool add64 = l == 0 && acc;
      if (q.lv[l].pen[fam] && c->prec != STP_PREC_F64) {
        // the epilogue is a template parameter of the pencil kernel (one site per level
        // holds one epilogue: the add into the output only on level 0 of the last H cycle)
        const int epi = add64 ? EPI_ADD64 : u.addout ? EPI_ADDTS : EPI_STORE;
        const int puty = c->prec == STP_PREC_F32 ? pencil_up_ty<float>(epi) : pencil_up_ty<bf16>(epi);
        u.tiles = int(pencil_tiles(q.lv[l + 1].n, puty));
        u.sb = kPencilSlabs;
        u.pk = q.lv[l].pk[fam];
        u.pd = q.lv[l].pd[fam];
        vc.upp[l].add(u, long(u.tiles) * ((q.N + u.sb - 1) / u.sb), true);
        vc.upp[l].epi = epi;
      } else {
        u.tiles = int(tiles_up_d(q.dim, q.lv[l].n));
        u.sb = sched_sb(u.tiles, q.N, (l == 0 && acc) ? c->sched.e[KN_UPA0] : c->sched.e[KN_UP0 + l]);
        vc.up[l].add(u, long(u.tiles) * ((q.N + u.sb - 1) / u.sb), u.op.cmode != CM_SLAB);
        vc.up[l].epi = (l == 0 && acc) ? EPI_ADD64 : EPI_STORE;
      }
    }
    FuseJob fj{};
    fj.S = q.N;
    fj.nlev = Lq - ft;
    for (int k = 0; k < fj.nlev; ++k) {
      fj.n[k] = q.lv[ft + k].n;
      fj.kap[k] = q.lv[ft + k].kscaled;
    }
    fj.op = family_op(q, ft, fam);
    fj.b = (ft == 0) ? T.in : q.lv[ft].b;
    fj.out = (ft == 0) ? T.out : q.lv[ft].e;
    fj.acc64 = (ft == 0) ? T.acc64 : nullptr;
    fj.addout = (ft == 0 && addout) ? 1 : 0;
    fj.state = &q.state->done;
    Site<FuseJob>& fs = vc.fused[ft];
    fs.add(fj, q.N);
    fs.epi = (ft == 0 && acc) ? EPI_ADD64 : EPI_STORE;
    fs.shmem = std::max(fs.shmem, fuse_lds(q.dim, fj, tc_bytes(c->prec)));
    fs.threads = fuse_threads(c->sched.e[KN_FUSE]);
  }
}

int fft2_l1(int N) {
  int L1 = 0;
  while ((1 << (2 * L1)) < N) ++L1;   // N1 = 2^ceil(log2(N)/2)
  return L1;
}

// transform path of a site: the dense group, a tuned choice, or the default
void site_path(stp_ctx* c, Site<TimeJob>& s) {
  const size_t tcb = tc_bytes(c->prec);
  s.C = 0;
  s.lds = 0;
  if (s.key < 0) {
    s.path = TP_DENSE;
    return;
  }
  auto it = c->sched.tpath.find(s.key);
  if (it != c->sched.tpath.end()) {
    s.path = it->second.path;
    s.C = it->second.C;
  } else if (s.key >= kBlueKey) {
    const int M = s.key - kBlueKey;
    s.path = M <= 32 ? TP_DENSE : TP_BLUESTEIN;   // N <= 16: the dense sum is cheaper
    s.C = s.path == TP_BLUESTEIN ? bluestein_cols(M, tcb) : 0;
  } else {
    size_t lds;
    transform_path(s.key, tcb, s.path, s.C, lds);
  }
  if (s.path == TP_STOCKHAM) s.lds = stockham_lds(s.key, s.C, tcb);
  if (s.path == TP_BLUESTEIN) s.lds = bluestein_lds(s.key - kBlueKey, s.C, tcb);
  if (s.path == TP_FOUR) s.lds = four_lds(s.key, s.C, tcb);
}

void build_transforms(stp_ctx* c, std::vector<Site<TimeJob>>& sites, int mode, const std::vector<const void*>& in,
                      const std::vector<void*>& out, const std::vector<double*>& acc64,
                      const std::vector<double>& alpha) {
  sites.clear();
  for (size_t i = 0; i < c->pr.size(); ++i) {
    if (!act(c, i)) continue;
    Problem& q = c->pr[i];
    // one site per power-of-two step count up to 4096, one per Bluestein
    // length M, and one dense site for the rest
    const int key = transform_key(q.N);
    Site<TimeJob>* s = nullptr;
    for (auto& t : sites)
      if (t.key == key) s = &t;
    if (!s) {
      sites.emplace_back();
      s = &sites.back();
      s->key = key;
      s->epi = (mode == 1) ? 1 : 0;
      site_path(c, *s);
    }
    TimeJob j{};
    j.npts = q.g0.npts;
    j.N = q.N;
    j.tw = q.tw;
    j.tw4 = q.tw4;
    j.M = q.blM;
    j.chirp = q.chirp;
    j.bhat = q.bhat;
    j.T = mode == 0 ? q.sinT : q.sinM;
    j.fs = q.fs;
    j.in = in[i];
    j.out = out[i];
    j.acc64 = acc64[i];
    j.alpha = alpha[i];
    j.state = &q.state->done;
    long nb;
    if (s->path == TP_FFT2) {
      const int Cc = kBlock >> fft2_l1(q.N);
      nb = (j.npts + Cc - 1) / Cc;
    } else if (s->path == TP_STOCKHAM || s->path == TP_BLUESTEIN) {
      nb = (j.npts + s->C - 1) / s->C;
    } else if (s->path == TP_FOUR) {
      nb = ((j.npts + s->C - 1) / s->C) * four_n1(q.N);
    } else {
      j.bx = int((j.npts + 63) / 64);
      nb = long(j.bx) * ((q.N + 4 * kDstKpt - 1) / (4 * kDstKpt));
    }
    s->add(j, nb);
  }
}

void build_sites(stp_ctx* c, const std::vector<double*>& u, const std::vector<double*>& p) {
  Sites& S = c->sites;
  const size_t P = c->pr.size();
  for (int w = 0; w < 2; ++w) {
    S.resid[w] = Site<ResidJob>();
    S.resid[w].threads = c->dim == 3 ? ResidTile<3>::threads : kBlock;
    for (size_t i = 0; i < P; ++i) {
      if (!act(c, i)) continue;
      Problem& q = c->pr[i];
      ResidJob j{};
      j.tiles = int(q.resid_tiles);
      j.sb = sched_sb(q.resid_tiles, q.N, c->sched.e[w == 0 ? KN_R0 : KN_R1]);
      const long nb = q.resid_tiles * ((q.N + j.sb - 1) / j.sb);
      if (w == 1) q.npart = nb;
      j.g = q.g0;
      j.t = TimeOp{q.kap64, q.cA64, q.R, q.N};
      j.taus = q.taus64;
      j.u = u[i];
      j.p = p[i];
      j.F = q.F;
      j.u0 = q.u0;
      j.r = q.W1;
      j.partial = q.partial;
      j.state = &q.state->done;
      S.resid[w].add(j, nb, q.R == 1);
    }
  }
  std::vector<VTop> topA(P), topH(P);
  std::vector<const void*> in4(P), in6(P);
  std::vector<void*> out4(P), out6(P, nullptr);
  std::vector<double*> acc4(P, nullptr), acc6(P);
  for (size_t i = 0; i < P; ++i) {
    Problem& q = c->pr[i];
    topA[i] = VTop{q.W1, nullptr, p[i]};       // p += A~^{-1} r_p
    topH[i] = VTop{q.W2, q.W1, nullptr};       // x = H~_k^{-1} rhat,  yhat = H~_k^{-1} y   (W2 -> W1)
    in4[i] = q.W1;                             // rhat = Phi^{-T} r_u   (W1 -> W2)
    out4[i] = q.W2;
    in6[i] = q.W1;                             // u += omega Phi^{-1} yhat
    acc6[i] = u[i];
  }
  build_vcycle(c, S.vc[VC_A], 0, topA, true);    // the A-tilde cycle adds into p
  build_vcycle(c, S.vc[VC_H1], 1, topH, false);  // the H cycles store
  build_vcycle(c, S.vc[VC_H2], 1, topH, false);
  S.vc[VC_AX] = VCycle();
  S.vc[VC_HX] = VCycle();
  S.vc[VC_HA] = VCycle();
  S.nures = Site<TileJob>();
  S.nu[0] = Site<TileJob>();
  S.nu[1] = Site<TileJob>();
  S.nu[0].threads = S.nu[1].threads = c->dim == 3 ? MidTile<3>::threads : kBlock;
  if (multi_cycle(c)) {
    std::vector<VTop> topAX(P), topHX(P);
    for (size_t i = 0; i < P; ++i) {
      Problem& q = c->pr[i];
      topAX[i] = VTop{q.W1, q.Xnu, nullptr};
      topHX[i] = VTop{q.W2, q.Xnu, nullptr};
      if (!act(c, i)) continue;
      // the operator tiles: b -= L x on the last cycle's correction x, and the
      // output so far takes x (A: the float64 p, bound per solve; H: o)
      TileJob j{};
      j.gf = q.g0;
      j.b = q.Xnu;
      j.addout = -1;
      j.state = &q.state->done;
      j.tiles = int(tiles_mid_d(q.dim, q.n));
      j.sb = sched_sb(j.tiles, q.N, c->sched.e[KN_MID]);
      const long nb = long(j.tiles) * ((q.N + j.sb - 1) / j.sb);
      j.op = family_op(q, 0, 0);
      j.out = q.W1;
      j.acc64 = p[i];
      S.nu[0].add(j, nb, j.op.cmode != CM_SLAB);
      j.op = family_op(q, 0, 1);
      j.out = q.W2;
      j.acc64 = nullptr;
      j.acc_ts = q.W1;
      S.nu[1].add(j, nb, j.op.cmode != CM_SLAB);
    }
    build_vcycle(c, S.vc[VC_AX], 0, topAX, false);
    build_vcycle(c, S.vc[VC_HX], 1, topHX, false);
    build_vcycle(c, S.vc[VC_HA], 1, topH, false, true);
    for (size_t i = 0; i < P; ++i) {
      if (!act(c, i)) continue;
      Problem& q = c->pr[i];
      TileJob j{};
      j.gf = q.g0;
      j.op = family_op(q, 0, 1);
      j.b = q.W1;                                // o, the first cycle's result
      j.out = q.W2;                              // the cycles' right-hand side, reduced in place
      j.addout = -1;
      j.state = &q.state->done;
      j.tiles = int(tiles_mid_d(q.dim, q.n));
      j.sb = sched_sb(j.tiles, q.N, c->sched.e[KN_MID]);
      S.nures.add(j, long(j.tiles) * ((q.N + j.sb - 1) / j.sb), j.op.cmode != CM_SLAB);
    }
  }
  S.mid = Site<TileJob>();
  S.mid.threads = S.nures.threads = c->dim == 3 ? MidTile<3>::threads : kBlock;
  for (size_t i = 0; i < P; ++i) {
    if (!act(c, i)) continue;
    Problem& q = c->pr[i];
    TileJob j{};
    j.gf = q.g0;
    j.op = family_op(q, 0, 2);
    j.b = q.W1;                                // y = (2/N) tau A x   (W1 -> W2)
    j.out = q.W2;
    j.state = &q.state->done;
    j.tiles = int(tiles_mid_d(q.dim, q.n));
    j.sb = sched_sb(j.tiles, q.N, c->sched.e[KN_MID]);
    S.mid.add(j, long(j.tiles) * ((q.N + j.sb - 1) / j.sb), j.op.cmode != CM_SLAB);
  }
  std::vector<double> one(P, 1.0), om(P);
  for (size_t i = 0; i < P; ++i) om[i] = c->pr[i].omega;
  build_transforms(c, S.a4, 0, in4, out4, acc4, one);
  build_transforms(c, S.a6, 1, in6, out6, acc6, om);
  S.fin.clear();
  for (size_t i = 0; i < P; ++i) {
    if (!act(c, i)) continue;
    Problem& q = c->pr[i];
    // finite elements: the a3 residual writes one partial per block of its (points, slabs) grid
    const long np = c->disc == STP_DISC_FEM ? q.nfnorm : q.npart;
    S.fin.push_back(FinJob{q.partial, np, q.state, c->opt.tol, c->opt.max_iter});
  }
}

template <typename J>
size_t site_bytes(const Site<J>& s) {
  return ((s.jobs.size() * sizeof(J)) + 255) & ~size_t(255);
}

template <typename F>
void for_each_site(Sites& S, F&& f) {
  f(S.resid[0]);
  f(S.resid[1]);
  for (auto& v : S.vc) {
    for (auto& x : v.down) f(x);
    for (auto& x : v.downp) f(x);
    for (auto& x : v.upp) f(x);
    for (auto& x : v.up) f(x);
    for (auto& x : v.fused) f(x);
    f(v.tri);
  }
  f(S.mid);
  f(S.nu[0]);
  f(S.nu[1]);
  f(S.nures);
  for (auto& x : S.a4) f(x);
  for (auto& x : S.a6) f(x);
}

size_t tables_bytes(Sites& S) {
  size_t b = 0;
  for_each_site(S, [&](auto& s) { b += site_bytes(s); });
  b += ((S.fin.size() * sizeof(FinJob)) + 255) & ~size_t(255);
  return b;
}

// every launch within the 32-bit work-item count of a dispatch
bool sites_fit(stp_ctx* c) {
  bool ok = true;
  for_each_site(c->sites, [&](auto& s) {
    if (double(s.blocks) * std::max(s.threads, kBlock) > 4294967295.0) ok = false;
    if (s.shmem > 65536) ok = false;   // fused multigrid launches stay within the default LDS limit
  });
  return ok;
}

void carve_tables(Sites& S, char* base) {
  size_t off = 0;
  for_each_site(S, [&](auto& s) {
    using J = typename std::decay<decltype(s.jobs[0])>::type;
    s.dev = s.jobs.empty() ? nullptr : reinterpret_cast<J*>(base + off);
    off += site_bytes(s);
  });
  S.fin_dev = reinterpret_cast<FinJob*>(base + off);
}

template <typename J>
stp_status upload_site(stp_ctx* c, Site<J>& s) {
  if (s.jobs.empty()) return STP_OK;
  HIP_TRY(hipMemcpyAsync(s.dev, s.jobs.data(), s.jobs.size() * sizeof(J), hipMemcpyHostToDevice, c->stream));
  return STP_OK;
}

stp_status upload_all(stp_ctx* c) {
  stp_status st = STP_OK;
  for_each_site(c->sites, [&](auto& s) {
    if (st == STP_OK) st = upload_site(c, s);
  });
  if (st != STP_OK) return st;
  HIP_TRY(hipMemcpyAsync(c->sites.fin_dev, c->sites.fin.data(), c->sites.fin.size() * sizeof(FinJob),
                         hipMemcpyHostToDevice, c->stream));
  return STP_OK;
}

// Point the per-solve jobs at device vectors: the residual launches read u,
// p (and f built from F, u0; Fz, when given, replaces both by another
// vector of the problem's size), the A-tilde cycle accumulates into acc_p,
// and the inverse transform accumulates alpha * Phi^{-1} yhat into acc_u
// (alpha < 0: each problem's omega).  Tables are uploaded on the context's
// stream.
stp_status bind_jobs(stp_ctx* c, const std::vector<double*>& u, const std::vector<double*>& p,
                     const std::vector<double*>* Fz, const std::vector<double*>& acc_p,
                     const std::vector<double*>& acc_u, double alpha) {
  Sites& S = c->sites;
  const size_t P = c->pr.size();
  auto owner = [&](const int* st) -> size_t {
    for (size_t i = 0; i < P; ++i)
      if (st == &c->pr[i].state->done) return i;
    return 0;
  };
  for (int w = 0; w < 2; ++w)
    for (auto& j : S.resid[w].jobs) {
      const size_t i = owner(j.state);
      j.u = u[i];
      j.p = p[i];
      j.F = Fz ? (*Fz)[i] : c->pr[i].F;
      j.u0 = Fz ? (*Fz)[i] : c->pr[i].u0;
    }
  VCycle& A = S.vc[VC_A];
  if (!A.up.empty())
    for (auto& j : A.up[0].jobs) j.acc64 = acc_p[owner(j.state)];
  if (!A.upp.empty())
    for (auto& j : A.upp[0].jobs) j.acc64 = acc_p[owner(j.state)];
  if (!A.fused.empty())
    for (auto& j : A.fused[0].jobs) j.acc64 = acc_p[owner(j.state)];
  for (auto& j : A.tri.jobs) j.acc64 = acc_p[owner(j.state)];
  for (auto& j : S.nu[0].jobs) j.acc64 = acc_p[owner(j.state)];
  for (auto& s : S.a6)
    for (auto& j : s.jobs) {
      const size_t i = owner(j.state);
      j.acc64 = acc_u[i];
      j.alpha = alpha < 0 ? c->pr[i].omega : alpha;
    }
  stp_status st;
  if (c->disc == STP_DISC_FEM) {   // single problem: the vectors the FEM kernels read when they run
    Problem& q = c->pr[0];
    const FemBind fb{u[0], p[0], Fz ? (*Fz)[0] : q.F, Fz ? (*Fz)[0] : q.u0, acc_p[0]};
    HIP_TRY(hipMemcpyAsync(q.fbind, &fb, sizeof(FemBind), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if ((st = upload_site(c, S.resid[0])) != STP_OK) return st;
  if ((st = upload_site(c, S.resid[1])) != STP_OK) return st;
  if (!A.up.empty() && (st = upload_site(c, A.up[0])) != STP_OK) return st;
  if (!A.upp.empty() && (st = upload_site(c, A.upp[0])) != STP_OK) return st;
  if (!A.fused.empty() && (st = upload_site(c, A.fused[0])) != STP_OK) return st;
  if ((st = upload_site(c, A.tri)) != STP_OK) return st;
  if ((st = upload_site(c, S.nu[0])) != STP_OK) return st;
  for (auto& s : S.a6)
    if ((st = upload_site(c, s)) != STP_OK) return st;
  return STP_OK;
}

stp_status bind_solution(stp_ctx* c, const std::vector<double*>& u, const std::vector<double*>& p,
                         const std::vector<double*>& acc, double alpha) {
  return bind_jobs(c, u, p, nullptr, p, acc, alpha);
}


stp_status validate_one(const stp_grid* g, int N, double tau, const stp_kappa* kappa, const double* F,
                        const double* u0, const stp_options* opt) {
  if (!g || !kappa) return fail(STP_EINVAL, "NULL grid or kappa");
  if (g->dim < 1 || g->dim > 3) return fail(STP_EINVAL, "dim must be 1, 2 or 3 (got %d)", g->dim);
  if (g->n < 1) return fail(STP_EINVAL, "n must be >= 1 (got %d)", g->n);
  if (N < 1) return fail(STP_EINVAL, "N must be >= 1 (got %d)", N);
  if (!(tau > 0) || !std::isfinite(tau)) return fail(STP_EINVAL, "tau must be finite and > 0");
  if (kappa->rank < 1 || kappa->rank > STP_MAX_RANK) return fail(STP_EINVAL, "kappa rank must be 1..%d", STP_MAX_RANK);
  if (!kappa->fields || !kappa->tcoef) return fail(STP_EINVAL, "NULL kappa fields or tcoef");
  if (!F || !u0) return fail(STP_EINVAL, "NULL F or u0");
  if (opt->spatial == STP_SPATIAL_EXACT && g->dim != 1) return fail(STP_EUNSUPPORTED, "exact spatial solves are 1-D only");
  const long npts = ipow(g->n, g->dim);
  if (double(npts) * double(N) > 4.0e12 || npts > (1L << 31) - 1) return fail(STP_EINVAL, "problem too large");
  return STP_OK;
}

stp_status validate_opts(const stp_options* opt) {
  if (opt->precision < STP_PREC_F64 || opt->precision > STP_PREC_BF16) return fail(STP_EINVAL, "bad precision");
  if (opt->spatial < STP_SPATIAL_AUTO || opt->spatial > STP_SPATIAL_NONE) return fail(STP_EINVAL, "bad spatial mode");
  if (opt->nu_A < 1 || opt->nu_A > kMaxNu || opt->nu_H < 1 || opt->nu_H > kMaxNu)
    return fail(STP_EINVAL, "nu_A and nu_H must lie in 1..%d", kMaxNu);
  if (!(opt->tol >= 0)) return fail(STP_EINVAL, "tol must be >= 0");
  if (opt->max_iter < 0) return fail(STP_EINVAL, "max_iter must be >= 0");
  if (opt->disc != STP_DISC_FD && opt->disc != STP_DISC_FEM) return fail(STP_EINVAL, "bad discretisation %d", opt->disc);
  if (opt->disc == STP_DISC_FEM && (opt->nu_A != 1 || opt->nu_H != 1))
    return fail(STP_EUNSUPPORTED, "finite elements run one V-cycle per spatial solve (nu_A = nu_H = 1)");
  if (opt->sweeps < 0 || opt->sweeps > 4) return fail(STP_EINVAL, "sweeps must lie in 0..4");
  return STP_OK;
}

// ---------------------------------------------------------------------------
// automatic damping parameter
//
// Theorem 3.1 gives convergence for omega lambda_max < 2 (1 - rho_A)/(1 + rho_A)
// (eq. (3.7)), with lambda_max the largest eigenvalue of H~^{-1} S and rho_A
// the contraction of A~^{-1}; Theorem 4.1 bounds the eigenvalues through the
// constant alpha of eq. (2.2), too loosely to choose omega from.  The library
// estimates instead, with the iteration's own launches and for every problem
// of the batch at once:
//   * lambda_min, lambda_max of H~^{-1} S~, S~ = K^T A~^{-1} K + K + K^T + A
//     (what one sweep of eq. (3.1) applies to u with p restarted from zero and
//     f = 0), as the extreme Ritz values of kLanczosSteps steps of conjugate
//     gradients on S~ preconditioned by H~^{-1} (the Lanczos matrix of the CG
//     coefficients);
//   * rho_A by kPowerSteps power steps on I - A~^{-1} A.
// omega = min(0.95 * 2/(lambda_min + lambda_max), 0.9 * 2/lambda_max): the
// damping that balances the two spectral ends of the preconditioned
// Richardson limit (rho_A -> 0), kept clear of the limit 2/lambda_max that
// (3.7) tends to.  (3.7) itself is much tighter than needed with the rho_A of
// one V-cycle and is not imposed.  Start vectors: SplitMix64 at the index.
// ---------------------------------------------------------------------------
constexpr int kLanczosSteps = 12;
constexpr int kPowerSteps = 8;
constexpr unsigned long long kSeedLanczos = 0x5EEDull;
constexpr unsigned long long kSeedPower = 0xA5EEDull;

// eigenvalue k (0-based, ascending) of the symmetric tridiagonal (d, e), by
// bisection on Sturm counts (Givens' method)
double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int k) {
  const int m = int(d.size());
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {   // Gershgorin interval
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) > k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

stp_status estimate_omega(stp_ctx* c) {
  const size_t P = c->pr.size();
  bool any = false;
  for (auto& q : c->pr) any = any || q.omega_auto;
  if (!any) return STP_OK;
  std::vector<long> nv(P);
  size_t total = 0;
  for (size_t i = 0; i < P; ++i) {
    nv[i] = long(c->pr[i].N) * c->pr[i].g0.npts;
    total += size_t(5) * nv[i];
  }
  const size_t scal = P * (kDotBlocks + 1);
  double* mem = nullptr;
  bool owned = false;
  stp_status s0 = scratch_get(c, total + scal, &mem, &owned);
  if (s0 != STP_OK) return s0;
  std::vector<double*> r(P), z(P), d(P), q(P), pb(P);
  {
    size_t off = 0;
    for (size_t i = 0; i < P; ++i) {
      r[i] = mem + off;
      z[i] = r[i] + nv[i];
      d[i] = z[i] + nv[i];
      q[i] = d[i] + nv[i];
      pb[i] = q[i] + nv[i];
      off += size_t(5) * nv[i];
    }
  }
  double* part = mem + total;
  double* slots = part + P * kDotBlocks;
  std::vector<double> hslots(P);
  auto grid = [](long n) { return dim3(unsigned((n + kBlock - 1) / kBlock)); };
  auto body = [&]() -> stp_status {
    for (size_t i = 0; i < P; ++i) {   // every launch runs: stop flags cleared
      c->state_host[i] = DevState{};
      c->state_host[i].fnorm = c->pr[i].fnorm;
      HIP_TRY(hipMemcpyAsync(c->pr[i].state, &c->state_host[i], sizeof(DevState), hipMemcpyHostToDevice, c->stream));
    }
    // per-problem dots a_i . b_i, returned on the host
    auto dots = [&](const std::vector<double*>& a, const std::vector<double*>& b) -> stp_status {
      for (size_t i = 0; i < P; ++i) {
        KLAUNCH(k_dot_partial, dim3(kDotBlocks), dim3(kBlock), 0, c->stream, nv[i], (const double*)a[i],
                (const double*)b[i], part + i * kDotBlocks);
        LAUNCH_CHECK();
        KLAUNCH(k_sum_to, dim3(1), dim3(kBlock), 0, c->stream, (const double*)(part + i * kDotBlocks),
                long(kDotBlocks), slots + i);
        LAUNCH_CHECK();
      }
      HIP_TRY(hipMemcpyAsync(hslots.data(), slots, P * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      return STP_OK;
    };
    auto axpby = [&](size_t i, double a, const double* x, double b, double* y) -> stp_status {
      KLAUNCH(k_axpby, grid(nv[i]), dim3(kBlock), 0, c->stream, nv[i], a, x, b, y);
      LAUNCH_CHECK();
      return STP_OK;
    };
    // z_i = H~^{-1} x_i
    auto precH = [&](const std::vector<double*>& x, const std::vector<double*>& zz) -> stp_status {
      stp_status st;
      for (size_t i = 0; i < P; ++i) {
        if ((st = c->impl->cast_in(x[i], c->pr[i].W1, nv[i])) != STP_OK) return st;
        HIP_TRY(hipMemsetAsync(zz[i], 0, size_t(nv[i]) * 8, c->stream));
      }
      if ((st = bind_jobs(c, zz, zz, nullptr, zz, zz, 1.0)) != STP_OK) return st;
      return c->impl->run_precH();
    };
    // q_i = S~ x_i (pb, q: scratch; q doubles as the zero source while the residuals run)
    auto stilde = [&](const std::vector<double*>& x) -> stp_status {
      stp_status st;
      for (size_t i = 0; i < P; ++i) {
        HIP_TRY(hipMemsetAsync(q[i], 0, size_t(nv[i]) * 8, c->stream));
        HIP_TRY(hipMemsetAsync(pb[i], 0, size_t(nv[i]) * 8, c->stream));
      }
      if ((st = bind_jobs(c, x, pb, &q, pb, q, 1.0)) != STP_OK) return st;
      if ((st = c->impl->resid(0)) != STP_OK) return st;         // W1 = K x
      if ((st = c->impl->run_vcycle(VC_A)) != STP_OK) return st;  // pb = A~^{-1} K x
      if ((st = c->impl->resid(1)) != STP_OK) return st;         // W1 = -K^T pb - (K + K^T + A) x
      for (size_t i = 0; i < P; ++i)
        if ((st = c->impl->cast_out(c->pr[i].W1, -1.0, q[i], nv[i])) != STP_OK) return st;
      return STP_OK;
    };
    stp_status st;
    // conjugate gradients on S~ with preconditioner H~^{-1}
    for (size_t i = 0; i < P; ++i) {
      KLAUNCH(k_fill_pm1, grid(nv[i]), dim3(kBlock), 0, c->stream, nv[i], kSeedLanczos, r[i]);
      LAUNCH_CHECK();
    }
    if ((st = precH(r, z)) != STP_OK) return st;
    for (size_t i = 0; i < P; ++i) HIP_TRY(hipMemcpyAsync(d[i], z[i], size_t(nv[i]) * 8, hipMemcpyDeviceToDevice, c->stream));
    if ((st = dots(r, z)) != STP_OK) return st;
    std::vector<double> rz = hslots, rz0 = hslots;
    std::vector<std::vector<double>> al(P), be(P);
    std::vector<char> live(P, 1);
    for (int k = 0; k < kLanczosSteps; ++k) {
      if ((st = stilde(d)) != STP_OK) return st;
      if ((st = dots(d, q)) != STP_OK) return st;
      std::vector<double> a(P, 0.0);
      for (size_t i = 0; i < P; ++i) {
        if (live[i] && !(hslots[i] > 0 && std::isfinite(hslots[i]))) live[i] = 0;   // breakdown
        a[i] = live[i] ? rz[i] / hslots[i] : 0.0;
        if ((st = axpby(i, -a[i], q[i], 1.0, r[i])) != STP_OK) return st;
      }
      if ((st = precH(r, z)) != STP_OK) return st;
      if ((st = dots(r, z)) != STP_OK) return st;
      for (size_t i = 0; i < P; ++i) {
        if (!live[i]) continue;
        const double b = hslots[i] / rz[i];
        al[i].push_back(a[i]);
        be[i].push_back(b);
        rz[i] = hslots[i];
        // an exhausted Krylov space (tiny problems) ends that problem's steps
        if (!(hslots[i] > 1e-28 * rz0[i]) || !std::isfinite(b)) live[i] = 0;
        if ((st = axpby(i, 1.0, z[i], b, d[i])) != STP_OK) return st;
      }
    }
    // power steps e <- e - A~^{-1} A e (r reused as e; q is the zero u and f)
    for (size_t i = 0; i < P; ++i) {
      KLAUNCH(k_fill_pm1, grid(nv[i]), dim3(kBlock), 0, c->stream, nv[i], kSeedPower, r[i]);
      LAUNCH_CHECK();
    }
    if ((st = dots(r, r)) != STP_OK) return st;
    for (size_t i = 0; i < P; ++i)
      if ((st = axpby(i, 1.0 / std::sqrt(hslots[i]), r[i], 0.0, r[i])) != STP_OK) return st;
    std::vector<double> ratio(P, 0.0);
    std::vector<char> plive(P, 1);
    for (int k = 0; k < kPowerSteps; ++k) {
      for (size_t i = 0; i < P; ++i) HIP_TRY(hipMemsetAsync(q[i], 0, size_t(nv[i]) * 8, c->stream));
      if ((st = bind_jobs(c, q, r, &q, r, q, 1.0)) != STP_OK) return st;
      if ((st = c->impl->resid(0)) != STP_OK) return st;         // W1 = -A e
      if ((st = c->impl->run_vcycle(VC_A)) != STP_OK) return st;  // e += A~^{-1} W1
      if ((st = dots(r, r)) != STP_OK) return st;
      for (size_t i = 0; i < P; ++i) {
        if (!plive[i]) continue;
        ratio[i] = std::sqrt(hslots[i]);
        if (!(ratio[i] > 1e-300)) {
          ratio[i] = 0.0;
          plive[i] = 0;
          continue;
        }
        if ((st = axpby(i, 1.0 / ratio[i], r[i], 0.0, r[i])) != STP_OK) return st;
      }
    }
    for (size_t i = 0; i < P; ++i) {
      Problem& pq = c->pr[i];
      if (!pq.omega_auto) continue;
      const int m = int(al[i].size());
      if (m == 0) return fail(STP_EDEVICE, "omega estimate: no conjugate-gradient step for problem %zu", i);
      std::vector<double> dg(m), off(std::max(0, m - 1));
      for (int k = 0; k < m; ++k) {
        dg[k] = 1.0 / al[i][k] + (k > 0 ? be[i][k - 1] / al[i][k - 1] : 0.0);
        if (k + 1 < m) off[k] = std::sqrt(be[i][k]) / al[i][k];
      }
      const double lmin = tridiag_eig(dg, off, 0), lmax = tridiag_eig(dg, off, m - 1);
      if (!(lmin > 0 && lmax >= lmin && std::isfinite(lmax)))
        return fail(STP_EDEVICE, "omega estimate failed for problem %zu (lambda %.3e..%.3e)", i, lmin, lmax);
      pq.est_lmin = lmin;
      pq.est_lmax = lmax;
      pq.est_rho = ratio[i];
      pq.omega = std::min(0.95 * 2.0 / (lmin + lmax), 0.9 * 2.0 / lmax);
    }
    return STP_OK;
  };
  const stp_status s = body();
  scratch_put(c, mem, owned);
  return s;
}

int resolve_spatial(int dim, int spatial) {
  if (spatial == STP_SPATIAL_AUTO) return dim == 1 ? STP_SPATIAL_EXACT : STP_SPATIAL_MG;
  return spatial;
}

// Describe the problems of a batch (host only; no device work).
stp_status describe(stp_ctx* c, int P, const stp_grid* grids, const int* N, const double* tau,
                    const stp_kappa* kappa, const double* const* F, const double* const* u0) {
  c->P = P;
  c->pr.assign(P, Problem());
  c->dim = grids[0].dim;
  c->spatial = resolve_spatial(c->dim, c->opt.spatial);
  int rmax = 1;
  for (int i = 0; i < P; ++i) {
    Problem& q = c->pr[i];
    q.dim = grids[i].dim;
    if (q.dim != c->dim) return fail(STP_EUNSUPPORTED, "all problems of a batch must have the same dimension");
    q.n = grids[i].n;
    q.N = N[i];
    q.tau = tau ? tau[i] : 0.0;
    q.R = kappa ? kappa[i].rank : 1;
    q.F = F ? F[i] : nullptr;
    q.u0 = u0 ? u0[i] : nullptr;
    q.fields = kappa ? kappa[i].fields : nullptr;
    rmax = std::max(rmax, q.R);
    stp_status s = build_levels(c->spatial, q);
    if (s != STP_OK) return s;
  }
  c->rm = rmax <= 1 ? 1 : (rmax <= 2 ? 2 : 4);
  if (c->disc == STP_DISC_FEM) {
    if (P != 1) return fail(STP_EUNSUPPORTED, "finite elements: single-problem contexts only");
    if (c->pr[0].R != 1) return fail(STP_EUNSUPPORTED, "finite elements: kappa must have rank 1 (a constant field)");
    if (c->spatial == STP_SPATIAL_MG && c->dim == 1)
      return fail(STP_EUNSUPPORTED, "finite elements in 1-D use exact spatial solves");
    if (c->spatial == STP_SPATIAL_MG && c->pr[0].n < 3)
      return fail(STP_EUNSUPPORTED, "finite-element multigrid needs n = 2^L - 1 >= 3");
  }
  return STP_OK;
}

size_t plan_all(stp_ctx* c, Bump& bp) {
  for (auto& q : c->pr) plan_problem(c->prec, c->spatial, q, bp, multi_cycle(c), c->disc == STP_DISC_FEM);
  std::vector<double*> nul(c->P, nullptr);
  build_sites(c, nul, nul);
  c->tables_off = (bp.off + 255) & ~size_t(255);
  c->tables_bytes = tables_bytes(c->sites);
  return c->tables_off + c->tables_bytes + 256;
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
  o->tau_steps = nullptr;
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

size_t stp_device_bytes_allocated(void) { return g_dev_bytes.load(); }

size_t stp_workspace_bytes_batch(int P, const stp_grid* grids, const int* N, const int* rank,
                                 const stp_options* opt) {
  if (P < 1 || !grids || !N || !rank || !opt) return 0;
  if (validate_opts(opt) != STP_OK) return 0;
  for (int i = 0; i < P; ++i) {
    if (grids[i].dim < 1 || grids[i].dim > 3 || grids[i].n < 1 || N[i] < 1 || rank[i] < 1 || rank[i] > STP_MAX_RANK)
      return 0;
    if (opt->spatial == STP_SPATIAL_EXACT && grids[i].dim != 1) return 0;
  }
  stp_ctx c;
  c.opt = *opt;
  c.prec = opt->precision;
  c.disc = opt->disc;
  std::vector<stp_kappa> kap(P);
  for (int i = 0; i < P; ++i) kap[i].rank = rank[i];
  if (describe(&c, P, grids, N, nullptr, kap.data(), nullptr, nullptr) != STP_OK) return 0;
  Bump bp;
  return ((plan_all(&c, bp) + 255) & ~size_t(255)) + scratch_doubles(&c) * 8;
}

size_t stp_workspace_bytes(const stp_grid* g, int N, int rank, const stp_options* opt) {
  return stp_workspace_bytes_batch(1, g, &N, &rank, opt);
}

stp_status stp_create_batch(stp_ctx** out, int P, const stp_grid* grids, const int* N, const double* tau,
                            const stp_kappa* kappa, const double* const* F, const double* const* u0,
                            const stp_options* opt_in, void* workspace, size_t ws_bytes, void* hip_stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return fail(STP_EINVAL, "NULL output context pointer");
  *out = nullptr;
  if (P < 1 || !grids || !N || !tau || !kappa || !F || !u0) return fail(STP_EINVAL, "NULL batch argument or P < 1");
  stp_options opt;
  if (opt_in) opt = *opt_in;
  else stp_default_options(&opt);
  stp_status s = validate_opts(&opt);
  if (s != STP_OK) return s;
  if (opt.kref_coef && P > 1) return fail(STP_EINVAL, "kref_coef must be NULL for a batch of more than one problem");
  // non-uniform steps (every problem's, one after the other): tau[i] is the
  // reference step of eq. (2.2), <= 0 for the mean of problem i's steps
  std::vector<double> tref(tau, tau + P);
  std::vector<long> toff(P, 0);
  if (opt.tau_steps) {
    long off = 0;
    for (int i = 0; i < P; ++i) {
      if (N[i] < 1) return fail(STP_EINVAL, "problem %d: N must be >= 1", i);
      toff[i] = off;
      double sum = 0;
      for (int n = 0; n < N[i]; ++n) {
        const double t = opt.tau_steps[off + n];
        if (!(t > 0) || !std::isfinite(t))
          return fail(STP_EINVAL, "tau_steps[%ld] (problem %d, step %d) must be finite and > 0", off + n, i, n);
        sum += t;
      }
      if (!(tref[i] > 0)) tref[i] = sum / N[i];
      off += N[i];
    }
  }
  for (int i = 0; i < P; ++i)
    if ((s = validate_one(&grids[i], N[i], tref[i], &kappa[i], F[i], u0[i], &opt)) != STP_OK) return s;
  std::unique_ptr<stp_ctx> c(new stp_ctx());
  c->opt = opt;
  c->prec = opt.precision;
  c->disc = opt.disc;
  c->stream = (hipStream_t)hip_stream;
  if ((s = describe(c.get(), P, grids, N, tref.data(), kappa, F, u0)) != STP_OK) return s;
  for (int i = 0; i < P; ++i) {
    Problem& q = c->pr[i];
    q.omega_auto = !(opt.omega > 0);
    q.omega = q.omega_auto ? 0.8 : opt.omega;   // replaced by the estimate below when automatic
    q.tcoef.assign(kappa[i].tcoef, kappa[i].tcoef + size_t(q.R) * q.N);
    if (opt.tau_steps) q.taus.assign(opt.tau_steps + toff[i], opt.tau_steps + toff[i] + q.N);
    else q.taus.assign(q.N, q.tau);
    q.abar.assign(q.R, 0.0);
    if (opt.kref_coef) {
      for (int r = 0; r < q.R; ++r) q.abar[r] = opt.kref_coef[r];
    } else if (opt.tau_steps) {   // step-weighted time mean: tau A_ref = (1/N) sum_n tau_n A_n
      double tsum = 0;
      for (int n = 0; n < q.N; ++n) tsum += q.taus[n];
      for (int r = 0; r < q.R; ++r) {
        double sum = 0;
        for (int n = 0; n < q.N; ++n) sum += q.taus[n] * q.tcoef[size_t(r) * q.N + n];
        q.abar[r] = sum / tsum;
      }
    } else {
      for (int r = 0; r < q.R; ++r) {
        double sum = 0;
        for (int n = 0; n < q.N; ++n) sum += q.tcoef[size_t(r) * q.N + n];
        q.abar[r] = sum / q.N;
      }
    }
  }
  Bump dry;
  const size_t need = plan_all(c.get(), dry);
  if (workspace) {   // [solver buffers | launch tables | setup and tuning scratch]
    const size_t soff = (need + 255) & ~size_t(255);
    const size_t sn = scratch_doubles(c.get());
    if (ws_bytes < soff + sn * 8)
      return fail(STP_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, soff + sn * 8);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(STP_EINVAL, "workspace not 256-byte aligned");
    c->ws = workspace;
    c->scratch = reinterpret_cast<double*>((char*)workspace + soff);
    c->scratch_n = sn;
  } else {   // the scratch is then allocated for the duration of each use
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(STP_ENOMEM, "hipMalloc of %zu bytes failed", need);
    }
    g_dev_bytes += need;
    c->own_ws = true;
  }
  Bump real;
  real.dry = false;
  real.base = (char*)c->ws;
  for (auto& q : c->pr) plan_problem(c->prec, c->spatial, q, real, multi_cycle(c.get()), c->disc == STP_DISC_FEM);
  HIP_TRY(hipHostMalloc((void**)&c->state_host, sizeof(DevState) * P, hipHostMallocDefault));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  switch (opt.precision) {
    case STP_PREC_F64: c->impl = make_solver_f64(c.get()); break;
    case STP_PREC_F32: c->impl = make_solver_f32(c.get()); break;
    default: c->impl = make_solver_bf16(c.get()); break;
  }
  if ((s = c->impl->init()) != STP_OK) return s;
  for (auto& q : c->pr) {
    if ((s = c->impl->setup_problem(q)) != STP_OK) return s;
    // kappa(t_n, x) > 0 at every node and step, and for the reference coefficient
    const long nn = q.g0.nnodes;
    const long nb = (nn + kBlock - 1) / kBlock;
    double* kscr = nullptr;
    bool owned = false;
    if ((s = scratch_get(c.get(), size_t(nb + kMaxRank), &kscr, &owned)) != STP_OK) return s;
    std::vector<double> cref(kMaxRank, 0.0);
    for (int r = 0; r < q.R; ++r) cref[r] = q.abar[r];
    double* part = kscr + kMaxRank;
    HIP_TRY(hipMemcpyAsync(kscr, cref.data(), kMaxRank * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<double> h(nb);
    double mn = 1e300;
    for (int pass = 0; pass < 2; ++pass) {
      KLAUNCH(k_kappa_min, dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, nn, q.R, pass == 0 ? q.N : 1, q.fields,
              pass == 0 ? (const double*)q.cA64 : (const double*)kscr, part);
      LAUNCH_CHECK();
      HIP_TRY(hipMemcpyAsync(h.data(), part, size_t(nb) * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      mn = std::min(mn, *std::min_element(h.begin(), h.end()));
    }
    double spread = 0.0, kap0 = 0.0;
    if (c->disc == STP_DISC_FEM) {   // the coefficient must be constant in space
      const long gb = std::min(nb, 512L);
      KLAUNCH(k_field_spread, dim3(unsigned(gb)), dim3(kBlock), 0, c->stream, nn, q.fields, part);
      LAUNCH_CHECK();
      HIP_TRY(hipMemcpyAsync(h.data(), part, size_t(gb) * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipMemcpyAsync(&kap0, q.fields, 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      spread = *std::max_element(h.begin(), h.begin() + gb);
    }
    scratch_put(c.get(), kscr, owned);
    if (!(mn > 0)) return fail(STP_EINVAL, "kappa must be > 0 at every node and step (min %.3e)", mn);
    if (c->disc == STP_DISC_FEM) {
      if (!(spread == 0.0)) return fail(STP_EINVAL, "finite elements: the kappa field must be constant in space");
      // element stencils of every level: the Galerkin operators of the coarse meshes, 2^-d per level
      q.fw.clear();
      for (size_t l = 0; l < q.lv.size(); ++l)
        q.fw.push_back(fem_stencils(q.dim, q.lv[l].n, kap0, std::ldexp(1.0, -int(q.dim * l))));
    }
    // ||f||
    const dim3 gr = grid_pts(q.g0.npts, q.N);
    if (c->disc == STP_DISC_FEM) {
      switch (q.dim) {
        case 1: KLAUNCH(k_fem_fnorm<1>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, fem_w64(q), (const double*)q.taus64, q.F, q.u0, q.partial); break;
        case 2: KLAUNCH(k_fem_fnorm<2>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, fem_w64(q), (const double*)q.taus64, q.F, q.u0, q.partial); break;
        default: KLAUNCH(k_fem_fnorm<3>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, fem_w64(q), (const double*)q.taus64, q.F, q.u0, q.partial);
      }
    } else {
      KLAUNCH(k_fnorm, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, (const double*)q.taus64, q.F, q.u0, q.partial);
    }
    LAUNCH_CHECK();
    KLAUNCH(k_sum_to, dim3(1), dim3(kBlock), 0, c->stream, (const double*)q.partial, q.nfnorm, &q.state->fnorm);
    LAUNCH_CHECK();
    DevState hs{};
    HIP_TRY(hipMemcpyAsync(&hs, q.state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    q.fnorm = std::sqrt(hs.fnorm);
    if (!std::isfinite(q.fnorm)) return fail(STP_EINVAL, "F or u0 holds a non-finite value");
  }
  // launch tables (jobs point at null u, p until a solve binds them)
  std::vector<double*> nul(P, nullptr);
  build_sites(c.get(), nul, nul);
  if (!sites_fit(c.get())) return fail(STP_EUNSUPPORTED, "a launch exceeds the dispatch size limit");
  if (tables_bytes(c->sites) > c->tables_bytes) return fail(STP_EDEVICE, "launch tables outgrew their reservation");
  carve_tables(c->sites, (char*)c->ws + c->tables_off);
  if ((s = upload_all(c.get())) != STP_OK) return s;
  if (c->spatial != STP_SPATIAL_NONE) {
    const auto te = std::chrono::steady_clock::now();
    if ((s = estimate_omega(c.get())) != STP_OK) return s;
    if (!(opt.omega > 0))   // estimated: the time it took (a given omega costs nothing)
      c->t_omega_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - te).count();
    build_sites(c.get(), nul, nul);   // f from F and u0 again; omega into the transform jobs
    if (tables_bytes(c->sites) > c->tables_bytes) return fail(STP_EDEVICE, "launch tables outgrew their reservation");
    carve_tables(c->sites, (char*)c->ws + c->tables_off);
    if ((s = upload_all(c.get())) != STP_OK) return s;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  *out = c.release();
  return STP_OK;
}

stp_status stp_create(stp_ctx** out, const stp_grid* g, int N, double tau, const stp_kappa* kappa, const double* F,
                      const double* u0, const stp_options* opt, void* workspace, size_t ws_bytes,
                      void* hip_stream) {
  if (!g || !kappa) {
    if (out) *out = nullptr;
    return fail(STP_EINVAL, "NULL grid or kappa");
  }
  return stp_create_batch(out, 1, g, &N, &tau, kappa, &F, &u0, opt, workspace, ws_bytes, hip_stream);
}

int stp_batch_size(stp_ctx* c) { return c ? c->P : 0; }

stp_status stp_omega_info(stp_ctx* c, int i, double* out5) {
  if (!c || !out5 || i < 0 || i >= c->P) return fail(STP_EINVAL, "bad context, problem index or output");
  const Problem& q = c->pr[i];
  out5[0] = q.omega;
  out5[1] = q.est_lmin;
  out5[2] = q.est_lmax;
  out5[3] = q.est_rho;
  // damping bound of eq. (3.7) from the estimates (0 when omega was given)
  out5[4] = q.est_lmax > 0 ? 2.0 * (1.0 - q.est_rho) / ((1.0 + q.est_rho) * q.est_lmax) : 0.0;
  return STP_OK;
}

stp_status stp_set_omega(stp_ctx* c, const double* omega) {
  if (!c || !omega) return fail(STP_EINVAL, "NULL argument");
  for (int i = 0; i < c->P; ++i)
    if (!(omega[i] > 0) || !std::isfinite(omega[i])) return fail(STP_EINVAL, "omega[%d] must be finite and > 0", i);
  for (int i = 0; i < c->P; ++i) c->pr[i].omega = omega[i];
  return STP_OK;   // taken into the launch tables when the next solve binds its vectors
}

stp_status stp_set_stop(stp_ctx* c, double tol, int max_iter) {
  if (!c) return fail(STP_EINVAL, "NULL context");
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(STP_EINVAL, "tol must be finite and >= 0");
  if (max_iter < 0) return fail(STP_EINVAL, "max_iter must be >= 0");
  c->opt.tol = tol;
  c->opt.max_iter = max_iter;
  for (auto& j : c->sites.fin) {
    j.tol = tol;
    j.max_iter = max_iter;
  }
  // the stop-test kernel reads these when it runs, so captured graphs stay valid
  HIP_TRY(hipMemcpyAsync(c->sites.fin_dev, c->sites.fin.data(), c->sites.fin.size() * sizeof(FinJob),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
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
  if (c->gexecA) (void)hipGraphExecDestroy(c->gexecA);
  if (c->gexecH) (void)hipGraphExecDestroy(c->gexecH);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

stp_status stp_apply_operator(stp_ctx* c, int op, const double* x, double* y) {
  if (!c || !x || !y) return fail(STP_EINVAL, "NULL argument");
  if (c->P != 1) return fail(STP_EUNSUPPORTED, "stp_apply_operator needs a single-problem context");
  Problem& q = c->pr[0];
  const dim3 gr = grid_pts(q.g0.npts, q.N);
  TimeOp t{q.kap64, q.cA64, q.R, q.N};
  const long nv = long(q.N) * q.g0.npts;
  if (c->disc == STP_DISC_FEM) {
    const FemW<double> w = fem_w64(q);
    const double* cA = q.cA64;
    const double* taus = q.taus64;
    if (op == STP_OP_B) {
      switch (c->dim) {
        case 1: KLAUNCH(k_fem_apply_B<1>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, cA, x, y); break;
        case 2: KLAUNCH(k_fem_apply_B<2>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, cA, x, y); break;
        default: KLAUNCH(k_fem_apply_B<3>, gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, cA, x, y);
      }
    } else if (op == STP_OP_SADDLE) {
      switch (c->dim) {
        case 1: KLAUNCH((k_fem_saddle<1, false>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, taus, cA, q.F, q.u0, x, x + nv, y, y + nv); break;
        case 2: KLAUNCH((k_fem_saddle<2, false>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, taus, cA, q.F, q.u0, x, x + nv, y, y + nv); break;
        default: KLAUNCH((k_fem_saddle<3, false>), gr, dim3(kBlock), 0, c->stream, q.g0, q.N, w, taus, cA, q.F, q.u0, x, x + nv, y, y + nv);
      }
    } else {
      return fail(STP_EINVAL, "unknown operator %d", op);
    }
    LAUNCH_CHECK();
    return STP_OK;
  }
  if (op == STP_OP_B) {
    switch (c->dim) {
      case 1: KLAUNCH(k_apply_B<1>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, y); break;
      case 2: KLAUNCH(k_apply_B<2>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, y); break;
      default: KLAUNCH(k_apply_B<3>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, y); break;
    }
  } else if (op == STP_OP_SADDLE) {
    switch (c->dim) {
      case 1: KLAUNCH(k_apply_saddle<1>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, x + nv, y, y + nv); break;
      case 2: KLAUNCH(k_apply_saddle<2>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, x + nv, y, y + nv); break;
      default: KLAUNCH(k_apply_saddle<3>, gr, dim3(kBlock), 0, c->stream, q.g0, t, x, x + nv, y, y + nv); break;
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
  if (c->P != 1) return fail(STP_EUNSUPPORTED, "stp_apply_precond needs a single-problem context");
  Problem& q = c->pr[0];
  const long nv = long(q.N) * q.g0.npts;
  // the stop flag must read "running" for the kernels to execute
  c->state_host[0] = DevState{};
  c->state_host[0].fnorm = q.fnorm;
  HIP_TRY(hipMemcpyAsync(q.state, &c->state_host[0], sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  stp_status s;
  // accumulate into z (A: the p target; H: the Phi^{-1} target with factor 1)
  std::vector<double*> zv(1, z);
  if ((s = bind_solution(c, zv, zv, zv, 1.0)) != STP_OK) return s;
  HIP_TRY(hipMemsetAsync(z, 0, size_t(nv) * 8, c->stream));
  if ((s = c->impl->cast_in(r, q.W1, nv)) != STP_OK) return s;
  s = which == STP_PC_A ? c->impl->run_vcycle(VC_A) : c->impl->run_precH();
  if (s != STP_OK) return s;
  HIP_TRY(hipStreamSynchronize(c->stream));   // the job tables are rebound by the next call
  return STP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// GMRES acceleration of the Uzawa sweep
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaxRestart = 64;
constexpr int kGsBlocks = 2048;   // blocks of the Gram-Schmidt reductions (fixed: deterministic sums)

// workspace of stp_gmres_solve, offsets in doubles, every region 256-byte aligned
struct GmresLayout {
  size_t v2 = 0;   // stride of the basis vectors (2 N n^d, rounded up)
  size_t V = 0, Z = 0, ucand = 0, part = 0, slots = 0, coef = 0, total = 0;
};

GmresLayout gmres_layout(const Problem& q, int m) {
  auto al = [](size_t x) { return (x + 31) & ~size_t(31); };
  const long nv = long(q.N) * q.g0.npts;
  const dim3 gp = grid_pts(q.g0.npts, q.N);
  const size_t fparts = size_t(gp.x) * gp.y * gp.z;
  GmresLayout L;
  L.v2 = al(size_t(2) * nv);
  L.V = 0;
  L.Z = L.V + size_t(m + 1) * L.v2;
  L.ucand = L.Z + size_t(m) * L.v2;
  L.part = L.ucand + al(nv);
  L.slots = L.part + al(std::max(size_t(kMaxRestart + 2) * kGsBlocks, fparts));
  L.coef = L.slots + al(2 * (kMaxRestart + 2));
  L.total = L.coef + al(kMaxRestart + 1);
  return L;
}

// ||r_p||^2 and ||r_u||^2 of the pair (u, p) of problem i into its state
// (rp2, ru2): one pass over u, p and F after a solve.
stp_status pair_norms(stp_ctx* c, int i, const double* u, const double* p) {
  Problem& q = c->pr[i];
  const TimeOp t{q.kap64, q.cA64, q.R, q.N};
  const long nb = std::max(1L, std::min(long(kNormBlocks), (q.g0.npts + kBlock - 1) / kBlock));
  c->kt.level = 0;
  if (c->disc == STP_DISC_FEM) {
    const FemW<double> w = fem_w64(q);
    switch (c->dim) {
      case 1: KLAUNCH(k_fem_saddle_norms<1>, dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, q.g0, q.N, w, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, q.nrm); break;
      case 2: KLAUNCH(k_fem_saddle_norms<2>, dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, q.g0, q.N, w, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, q.nrm); break;
      default: KLAUNCH(k_fem_saddle_norms<3>, dim3(unsigned(nb)), dim3(kBlock), 0, c->stream, q.g0, q.N, w, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, q.nrm);
    }
    LAUNCH_CHECK();
    KLAUNCH(k_sum_rows, dim3(2), dim3(kBlock), 0, c->stream, (const double*)q.nrm, nb, &q.state->rp2);
    LAUNCH_CHECK();
    return STP_OK;
  }
  // one job on the up-sweep's tiles (both operands staged per slab), slabs per
  // block as the default schedule
  const long ntl = tiles_up_d(q.dim, q.n);
  ResidJob j{};
  j.tiles = int(ntl);
  j.sb = sched_sb(ntl, q.N, 0);
  j.g = q.g0;
  j.t = t;
  j.taus = q.taus64;
  j.u = u;
  j.p = p;
  j.F = q.F;
  j.u0 = q.u0;
  j.partial = q.nrm;
  const long cnt = ntl * ((q.N + j.sb - 1) / j.sb);
  HIP_TRY(hipMemcpyAsync(q.njob, &j, sizeof(ResidJob), hipMemcpyHostToDevice, c->stream));
  const dim3 gr(static_cast<unsigned>(cnt)), bl(kBlock);
  const bool fix = q.R == 1;
  switch (c->dim * 10 + c->rm) {
#define STP_PN(D, RM)                                                                                 \
  case D * 10 + RM:                                                                                   \
    if (fix) KLAUNCH((k_pair_norms<D, 1, 1>), gr, bl, 0, c->stream, (const ResidJob*)q.njob, 1);      \
    else KLAUNCH((k_pair_norms<D, RM, 0>), gr, bl, 0, c->stream, (const ResidJob*)q.njob, 1);         \
    break;
    STP_PN(1, 1) STP_PN(1, 2) STP_PN(1, 4) STP_PN(2, 1) STP_PN(2, 2) STP_PN(2, 4) STP_PN(3, 1) STP_PN(3, 2)
    default: STP_PN(3, 4)
#undef STP_PN
  }
  LAUNCH_CHECK();
  KLAUNCH(k_sum_rows, dim3(2), dim3(kBlock), 0, c->stream, (const double*)q.nrm, cnt, &q.state->rp2);
  LAUNCH_CHECK();
  return STP_OK;
}

// Device time per phase of the timing records r0 .. r1-1 (0 unless timing is on).
void phase_times(stp_ctx* c, size_t r0, size_t r1, double* out) {
  for (int k = 0; k < PH_COUNT; ++k) out[k] = 0.0;
  if (!c->kt.on) return;
  for (size_t k = r0; k < r1 && k < c->kt.recs.size(); ++k) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->kt.recs[k].a, c->kt.recs[k].b) == hipSuccess) out[c->kt.recs[k].phase] += ms;
  }
}

// Capture the launches of body on a private stream (capture is not possible on
// the null stream) and instantiate them into *out.
stp_status capture_graph(stp_ctx* c, hipGraphExec_t* out, const std::function<stp_status()>& body) {
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  c->stream = c->cap_stream;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  stp_status s = STP_OK;
  if (e == hipSuccess) {
    s = body();
    e = hipStreamEndCapture(c->cap_stream, &graph);
  }
  c->stream = saved;
  if (s != STP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(STP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(STP_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  return STP_OK;
}

}  // namespace

extern "C" {

size_t stp_gmres_workspace_bytes(stp_ctx* c, int restart) {
  if (!c || c->P != 1 || restart < 1 || restart > kMaxRestart) return 0;
  return gmres_layout(c->pr[0], restart).total * 8;
}

}  // extern "C"

namespace {

// Arguments common to both GMRES entry points.
stp_status gmres_check(stp_ctx* c, double* u, double* p, int restart) {
  if (!c || !u || !p) return fail(STP_EINVAL, "NULL argument (u and p are required)");
  if (c->P != 1) return fail(STP_EUNSUPPORTED, "GMRES needs a single-problem context");
  if (c->spatial == STP_SPATIAL_NONE) return fail(STP_EUNSUPPORTED, "context created without a spatial solver");
  if (restart < 1 || restart > kMaxRestart) return fail(STP_EINVAL, "restart %d not in 1..%d", restart, kMaxRestart);
  return STP_OK;
}

// Flexible GMRES(restart) around the Uzawa sweep with its vectors at base
// (gmres_layout doubles).  graph: replay the two preconditioner solves as
// captured HIP graphs (captured on first use); false launches them eagerly.
stp_status gmres_run(stp_ctx* c, double* u, double* p, int restart, double* base, bool graph, double* hist,
                     stp_stats* stats) {
  Problem& q = c->pr[0];
  const GmresLayout L = gmres_layout(q, restart);
  const long nv = long(q.N) * q.g0.npts;
  const long v2 = long(L.v2);
  double* V = base + L.V;
  double* Z = base + L.Z;
  double* uc = base + L.ucand;
  double* part = base + L.part;
  double* slots = base + L.slots;
  double* coef = base + L.coef;
  const dim3 gp = grid_pts(q.g0.npts, q.N);
  const long fparts = long(gp.x) * gp.y * gp.z;
  const TimeOp t{q.kap64, q.cA64, q.R, q.N};
  // f = 0: the stop test and the reported residuals are absolute
  const double fnorm = q.fnorm > 0 ? q.fnorm : 1.0, gnorm = std::sqrt(2.0) * fnorm;
  const double omega = q.omega, tol = c->opt.tol;
  const int max_iter = c->opt.max_iter;
  auto vgrid = [](long n) { return dim3(unsigned((n + kBlock - 1) / kBlock)); };
  std::vector<double> hs(2 * (kMaxRestart + 2));

  // the tile kernels run only while the problem's stop flag reads "running"
  c->state_host[0] = DevState{};
  c->state_host[0].fnorm = q.fnorm;
  HIP_TRY(hipMemcpyAsync(q.state, &c->state_host[0], sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  const size_t rec0 = c->kt.recs.size();
  HIP_TRY(hipEventRecord(c->ev0, c->stream));

  // ||f - B uu||_2 (synchronises)
  const bool fem = c->disc == STP_DISC_FEM;
  const FemW<double> fw64 = fem ? fem_w64(q) : FemW<double>{};
  auto fmBu = [&](const double* uu, double& out) -> stp_status {
    if (fem) {
      switch (c->dim) {
        case 1: KLAUNCH(k_fem_fmBu_partial<1>, gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, uu, part); break;
        case 2: KLAUNCH(k_fem_fmBu_partial<2>, gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, uu, part); break;
        default: KLAUNCH(k_fem_fmBu_partial<3>, gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, uu, part);
      }
    } else switch (c->dim) {
      case 1: KLAUNCH(k_fmBu_partial<1>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, uu, part); break;
      case 2: KLAUNCH(k_fmBu_partial<2>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, uu, part); break;
      default: KLAUNCH(k_fmBu_partial<3>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, uu, part);
    }
    LAUNCH_CHECK();
    KLAUNCH(k_sum_rows, dim3(1), dim3(kBlock), 0, c->stream, (const double*)part, fparts, slots);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(hs.data(), slots, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out = std::sqrt(std::max(hs[0], 0.0));
    return STP_OK;
  };
  // out[0..k) = <V_i, w> (V_i = V + i v2), out[k] = <w, w> when self; device only
  auto mdot = [&](int k, const double* w, bool self, double* out) -> stp_status {
    for (int c0 = 0; c0 < k || (c0 == 0 && k == 0); c0 += kDotRows) {
      const int kk = std::min(kDotRows, k - c0);
      const bool last = c0 + kk >= k;
      KLAUNCH(k_mdot_partial, dim3(kGsBlocks), dim3(kBlock), 0, c->stream, 2 * nv, (const double*)(V + c0 * v2), v2,
              kk, int(self && last), w, part + long(c0) * kGsBlocks);
      LAUNCH_CHECK();
    }
    KLAUNCH(k_sum_rows, dim3(unsigned(k + (self ? 1 : 0))), dim3(kBlock), 0, c->stream, (const double*)part,
            long(kGsBlocks), out);
    LAUNCH_CHECK();
    return STP_OK;
  };
  auto maxpy = [&](double* w, long n, const double* Vb, int k, const double* cf, double sgn) -> stp_status {
    KLAUNCH(k_maxpy, vgrid(n), dim3(kBlock), 0, c->stream, n, w, Vb, v2, k, cf, sgn);
    LAUNCH_CHECK();
    return STP_OK;
  };
  // w -= sum_{i<k} cf[i] V_i over the whole saddle vector, then *out = ||w||^2 (device)
  auto project = [&](double* w, int k, const double* cf, double* out) -> stp_status {
    KLAUNCH(k_maxpy_norm, dim3(kGsBlocks), dim3(kBlock), 0, c->stream, 2 * nv, w, (const double*)V, v2, k, cf,
            part);
    LAUNCH_CHECK();
    KLAUNCH(k_sum_rows, dim3(1), dim3(kBlock), 0, c->stream, (const double*)part, long(kGsBlocks), out);
    LAUNCH_CHECK();
    return STP_OK;
  };
  auto scale = [&](double* x, long n, double a) -> stp_status {
    KLAUNCH(k_axpby, vgrid(n), dim3(kBlock), 0, c->stream, n, a, (const double*)x, 0.0, x);
    LAUNCH_CHECK();
    return STP_OK;
  };
  // z = P^{-1} v: one Uzawa sweep from zero, [A~^{-1} v_p; -omega H~^{-1}(v_u + K^T A~^{-1} v_p)].
  // The two solves replay captured graphs (they read the job tables, rebound
  // for every z, at replay time).
  if (graph && !c->gexecA) {
    stp_status s = capture_graph(c, &c->gexecA, [c]() { return c->impl->run_vcycle(VC_A); });
    if (s != STP_OK) return s;
  }
  if (graph && !c->gexecH) {
    stp_status s = capture_graph(c, &c->gexecH, [c]() { return c->impl->run_precH(); });
    if (s != STP_OK) return s;
  }
  auto precond = [&](const double* vj, double* zj) -> stp_status {
    stp_status s;
    HIP_TRY(hipMemsetAsync(zj, 0, size_t(2 * nv) * 8, c->stream));
    std::vector<double*> zp(1, zj), zu(1, zj + nv);
    if ((s = bind_jobs(c, zp, zp, nullptr, zp, zu, omega)) != STP_OK) return s;
    if ((s = c->impl->cast_in(vj, q.W1, nv)) != STP_OK) return s;
    c->kt.phase = PH_ATILDE;
    if (graph) HIP_TRY(hipGraphLaunch(c->gexecA, c->stream));             // z_p += A~^{-1} v_p
    else if ((s = c->impl->run_vcycle(VC_A)) != STP_OK) return s;
    c->kt.phase = PH_OTHER;
    if ((s = c->impl->kt_add_in(vj + nv, zj, -1.0)) != STP_OK) return s;  // W1 = -(v_u + K^T z_p)
    if (graph) HIP_TRY(hipGraphLaunch(c->gexecH, c->stream));             // z_u += omega H~^{-1} W1
    else if ((s = c->impl->run_precH()) != STP_OK) return s;
    return STP_OK;
  };
  // upper-triangular solve of the rotated Hessenberg system (host), then upload
  auto solve_y = [&](const std::vector<double>& H, const std::vector<double>& sv, int k, int m,
                     std::vector<double>& y) -> stp_status {
    y.assign(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double a = sv[i];
      for (int l = i + 1; l < k; ++l) a -= H[i * m + l] * y[l];
      y[i] = a / H[i * m + i];
    }
    HIP_TRY(hipMemcpyAsync(coef, y.data(), size_t(k) * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return STP_OK;
  };

  stp_status s;
  int iters = 0, nh = 0;
  int outcome = 3;   // 1 converged, 2 non-finite, 3 max_iter, 4 breakdown
  double res = 0.0;
  std::vector<double> H, cs, sn, sv, y;
  while (true) {
    if ((s = fmBu(u, res)) != STP_OK) return s;
    if (!std::isfinite(res)) { outcome = 2; break; }
    if (res <= tol * fnorm) { outcome = 1; break; }
    if (iters >= max_iter) break;
    const int m = std::min(restart, max_iter - iters);
    if (fem) switch (c->dim) {   // v_0 = g - S x
      case 1: KLAUNCH((k_fem_saddle<1, true>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, V, V + nv); break;
      case 2: KLAUNCH((k_fem_saddle<2, true>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, V, V + nv); break;
      default: KLAUNCH((k_fem_saddle<3, true>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, p, u, V, V + nv);
    }
    else switch (c->dim) {   // v_0 = g - S x
      case 1: KLAUNCH(k_saddle_resid<1>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, p, u, V, V + nv); break;
      case 2: KLAUNCH(k_saddle_resid<2>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, p, u, V, V + nv); break;
      default: KLAUNCH(k_saddle_resid<3>, gp, dim3(kBlock), 0, c->stream, q.g0, t, (const double*)q.taus64, q.F, q.u0, p, u, V, V + nv);
    }
    LAUNCH_CHECK();
    if ((s = mdot(0, V, true, slots)) != STP_OK) return s;
    HIP_TRY(hipMemcpyAsync(hs.data(), slots, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double beta = std::sqrt(std::max(hs[0], 0.0));
    if (hist && nh == 0) hist[nh++] = beta / gnorm;
    if (!(beta > 0.0)) { outcome = std::isfinite(beta) ? 1 : 2; break; }
    if ((s = scale(V, 2 * nv, 1.0 / beta)) != STP_OK) return s;
    H.assign(size_t(m + 1) * m, 0.0);
    cs.assign(m, 0.0);
    sn.assign(m, 0.0);
    sv.assign(m + 1, 0.0);
    sv[0] = beta;
    int k = 0;
    bool conv = false;
    for (int j = 0; j < m; ++j) {
      double* vj = V + j * v2;
      double* zj = Z + j * v2;
      double* w = V + (j + 1) * v2;
      if ((s = precond(vj, zj)) != STP_OK) return s;
      if (fem) switch (c->dim) {   // w = S z_j
        case 1: KLAUNCH((k_fem_saddle<1, false>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, zj, zj + nv, w, w + nv); break;
        case 2: KLAUNCH((k_fem_saddle<2, false>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, zj, zj + nv, w, w + nv); break;
        default: KLAUNCH((k_fem_saddle<3, false>), gp, dim3(kBlock), 0, c->stream, q.g0, q.N, fw64, (const double*)q.taus64, (const double*)q.cA64, q.F, q.u0, zj, zj + nv, w, w + nv);
      }
      else switch (c->dim) {   // w = S z_j
        case 1: KLAUNCH(k_apply_saddle<1>, gp, dim3(kBlock), 0, c->stream, q.g0, t, zj, zj + nv, w, w + nv); break;
        case 2: KLAUNCH(k_apply_saddle<2>, gp, dim3(kBlock), 0, c->stream, q.g0, t, zj, zj + nv, w, w + nv); break;
        default: KLAUNCH(k_apply_saddle<3>, gp, dim3(kBlock), 0, c->stream, q.g0, t, zj, zj + nv, w, w + nv);
      }
      LAUNCH_CHECK();
      // classical Gram-Schmidt, repeated once when the projection removes more
      // than 90 % of the norm (the orthogonality lost in one pass is about the
      // unit roundoff times the ratio of the norms before and after)
      if ((s = mdot(j + 1, w, true, slots)) != STP_OK) return s;
      if ((s = project(w, j + 1, slots, slots + (j + 2))) != STP_OK) return s;
      HIP_TRY(hipMemcpyAsync(hs.data(), slots, size_t(j + 3) * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      for (int i = 0; i <= j; ++i) H[i * m + j] = hs[i];
      double nn = hs[j + 2];
      if (nn < 1e-2 * hs[j + 1]) {
        if ((s = mdot(j + 1, w, false, slots)) != STP_OK) return s;
        if ((s = project(w, j + 1, slots, slots + (j + 1))) != STP_OK) return s;
        HIP_TRY(hipMemcpyAsync(hs.data(), slots, size_t(j + 2) * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int i = 0; i <= j; ++i) H[i * m + j] += hs[i];
        nn = hs[j + 1];
      }
      const double hn = std::sqrt(std::max(nn, 0.0));
      if (!std::isfinite(hn)) { outcome = 2; break; }
      if (hn > 0.0 && (s = scale(w, 2 * nv, 1.0 / hn)) != STP_OK) return s;
      for (int i = 0; i < j; ++i) {   // earlier rotations on the new column
        const double a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * b;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double hjj = H[j * m + j];
      const double den = std::hypot(hjj, hn);
      if (den == 0.0) break;   // singular least-squares problem
      cs[j] = hjj / den;
      sn[j] = hn / den;
      H[j * m + j] = den;
      sv[j + 1] = -sn[j] * sv[j];
      sv[j] = cs[j] * sv[j];
      k = j + 1;
      ++iters;
      const double est = std::fabs(sv[j + 1]);
      if (hist) hist[nh++] = est / gnorm;
      if (est <= tol * gnorm) {   // check the stop test on the candidate u
        if ((s = solve_y(H, sv, k, m, y)) != STP_OK) return s;
        HIP_TRY(hipMemcpyAsync(uc, u, size_t(nv) * 8, hipMemcpyDeviceToDevice, c->stream));
        if ((s = maxpy(uc, nv, Z + nv, k, coef, 1.0)) != STP_OK) return s;
        if ((s = fmBu(uc, res)) != STP_OK) return s;
        if (res <= tol * fnorm) {
          conv = true;
          break;
        }
      }
    }
    if (outcome == 2) break;
    if (k > 0) {   // x += Z y
      if ((s = solve_y(H, sv, k, m, y)) != STP_OK) return s;
      if ((s = maxpy(p, nv, Z, k, coef, 1.0)) != STP_OK) return s;
      if ((s = maxpy(u, nv, Z + nv, k, coef, 1.0)) != STP_OK) return s;
    }
    if (conv) { outcome = 1; break; }
    if (k == 0) { outcome = 4; break; }
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  const size_t r1 = c->kt.recs.size();
  c->kt.phase = PH_OTHER;
  if ((s = pair_norms(c, 0, u, p)) != STP_OK) return s;
  HIP_TRY(hipMemcpyAsync(&c->state_host[0], q.state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  const stp_status r = outcome == 1 ? STP_OK : outcome == 2 ? STP_EDIVERGED : STP_ENOTCONV;
  if (stats) {
    stats->iters = iters;
    stats->rel_res = res / fnorm;
    stats->omega_used = omega;
    stats->t_solve_ms = ms;
    stats->status = r;
    stats->rel_rp = std::sqrt(std::max(c->state_host[0].rp2, 0.0)) / fnorm;
    stats->rel_ru = std::sqrt(std::max(c->state_host[0].ru2, 0.0)) / fnorm;
    stats->t_setup_ms = c->t_setup_ms;
    stats->t_omega_ms = c->t_omega_ms;
    phase_times(c, rec0, r1, stats->t_phase_ms);
  }
  if (outcome == 2) return fail(r, "GMRES: non-finite residual after %d steps", iters);
  if (outcome == 4) return fail(r, "GMRES: breakdown after %d steps (rel %.3e)", iters, res / fnorm);
  if (outcome == 3) return fail(r, "GMRES: max_iter %d reached (rel %.3e)", max_iter, res / fnorm);
  return STP_OK;
}

// ---------------------------------------------------------------------------
// allocation-free GMRES: the Krylov vectors in a fixed device array of
// kScratchDoubles values.  Every device that runs the library holds its own
// copy of `scratch` until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device (the array's
// name in host code is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;   // device ordinal -> its copy of scratch

stp_status scratch_address(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {   // once per device, with that device current
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(STP_EDEVICE, "hipGetSymbolAddress of the fixed scratch failed: %s", hipGetErrorString(e));
    it = g_scratch_addr.emplace(dev, static_cast<double*>(ptr)).first;
  }
  *out = it->second;
  return STP_OK;
}

}  // namespace

extern "C" {

stp_status stp_gmres_solve_noalloc(stp_ctx* c, double* u, double* p, int restart, double* hist, stp_stats* stats) {
  stp_status s = gmres_check(c, u, p, restart);
  if (s != STP_OK) return s;
  const size_t need = gmres_layout(c->pr[0], restart).total;
  if (need > kScratchDoubles)
    return fail(STP_EINVAL, "GMRES(%d) of this problem needs %zu bytes; the fixed scratch holds %zu", restart,
                need * 8, kScratchDoubles * 8);
  double* base = nullptr;
  if ((s = scratch_address(&base)) != STP_OK) return s;
  // eager launches: instantiating a graph may allocate
  return gmres_run(c, u, p, restart, base, false, hist, stats);
}

stp_status stp_gmres_solve(stp_ctx* c, double* u, double* p, int restart, void* ws, size_t ws_bytes, double* hist,
                           stp_stats* stats) {
  stp_status s = gmres_check(c, u, p, restart);
  if (s != STP_OK) return s;
  const GmresLayout L = gmres_layout(c->pr[0], restart);
  if (!ws || ws_bytes < L.total * 8)
    return fail(STP_EINVAL, "GMRES workspace of %zu bytes given, %zu needed", ws_bytes, L.total * 8);
  if (reinterpret_cast<uintptr_t>(ws) % 8) return fail(STP_EINVAL, "GMRES workspace not 8-byte aligned");
  return gmres_run(c, u, p, restart, static_cast<double*>(ws), c->opt.use_graph && !c->kt.on, hist, stats);
}

// Capture one iteration over the batch on a private stream (capture is not
// possible on the null stream).  The graph reads the job tables at replay
// time, so it stays valid when a solve rebinds u and p.
static stp_status capture_iteration(stp_ctx* c) {
  if (c->gexec) return STP_OK;
  return capture_graph(c, &c->gexec, [c]() { return c->impl->iteration(); });
}

// Rebuild and upload the launch tables for the problems in c->active, bound to
// (u, p); the captured iteration graph has the old launch shapes and goes.
static stp_status retable(stp_ctx* c, const std::vector<double*>& u, const std::vector<double*>& p) {
  build_sites(c, u, p);
  if (tables_bytes(c->sites) > c->tables_bytes) return fail(STP_EDEVICE, "launch tables outgrew their reservation");
  carve_tables(c->sites, (char*)c->ws + c->tables_off);
  stp_status s = upload_all(c);
  if (s != STP_OK) return s;
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return STP_OK;
}

stp_status stp_uzawa_solve_batch(stp_ctx* c, double* const* u, double* const* p, stp_stats* stats) {
  if (!c || !u || !p) return fail(STP_EINVAL, "NULL argument");
  if (c->spatial == STP_SPATIAL_NONE) return fail(STP_EUNSUPPORTED, "context created without a spatial solver");
  std::vector<double*> uv(c->P), pv(c->P);
  for (int i = 0; i < c->P; ++i) {
    if (!u[i] || !p[i]) return fail(STP_EINVAL, "NULL u or p of problem %d (both are required)", i);
    uv[i] = u[i];
    pv[i] = p[i];
  }
  stp_status s;
  if (!c->active.empty()) {   // every problem back in the tables
    c->active.clear();
    if ((s = retable(c, uv, pv)) != STP_OK) return s;
  }
  for (int i = 0; i < c->P; ++i) {
    c->state_host[i] = DevState{};
    c->state_host[i].fnorm = c->pr[i].fnorm;
    HIP_TRY(hipMemcpyAsync(c->pr[i].state, &c->state_host[i], sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  }
  if ((s = bind_solution(c, uv, pv, uv, -1.0)) != STP_OK) return s;
  const bool graph = c->opt.use_graph && !c->kt.on;
  if (graph && (s = capture_iteration(c)) != STP_OK) return s;
  const size_t rec0 = c->kt.recs.size();
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  const int chunk = std::max(1, c->opt.check_every);
  const int max_launch = c->opt.max_iter + 1;   // iterations 0..max_iter each evaluate the stop test
  int launched = 0;
  while (true) {
    const int todo = std::min(chunk, max_launch - launched);
    for (int q = 0; q < todo; ++q) {
      // iteration max_iter always stops at its test: launch only its first half
      const bool last = launched == max_launch - 1;
      if (graph && !last) HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
      else if ((s = c->impl->iteration(!last)) != STP_OK) return s;
      ++launched;
    }
    for (int i = 0; i < c->P; ++i)
      HIP_TRY(hipMemcpyAsync(&c->state_host[i], c->pr[i].state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool all = true;
    for (int i = 0; i < c->P; ++i) all = all && c->state_host[i].done != 0;
    if (all) break;
    if (launched >= max_launch) return fail(STP_EDEVICE, "iteration state did not terminate");
    // batch: drop the problems that stopped since the last check from the tables
    bool dropped = false;
    for (int i = 0; i < c->P && c->P > 1; ++i) dropped = dropped || (act(c, i) && c->state_host[i].done != 0);
    if (dropped) {
      c->active.assign(c->P, 0);
      for (int i = 0; i < c->P; ++i) c->active[i] = c->state_host[i].done == 0;
      if ((s = retable(c, uv, pv)) != STP_OK) return s;
      if (graph && (s = capture_iteration(c)) != STP_OK) return s;
    }
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  const size_t r1 = c->kt.recs.size();
  if (!c->active.empty()) {   // full tables again for whatever runs next
    c->active.clear();
    if ((s = retable(c, uv, pv)) != STP_OK) return s;
  }
  c->kt.phase = PH_OTHER;
  for (int i = 0; i < c->P; ++i)   // residual blocks of the returned pairs (outside the timed loop)
    if ((s = pair_norms(c, i, uv[i], pv[i])) != STP_OK) return s;
  for (int i = 0; i < c->P; ++i)
    HIP_TRY(hipMemcpyAsync(&c->state_host[i], c->pr[i].state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  double tph[PH_COUNT];
  phase_times(c, rec0, r1, tph);   // the norm pass is not part of the solve's phases
  stp_status worst = STP_OK;
  for (int i = 0; i < c->P; ++i) {
    const DevState& hs = c->state_host[i];
    const stp_status r = hs.done == 1 ? STP_OK : (hs.done == 2 ? STP_EDIVERGED : STP_ENOTCONV);
    if (stats) {
      const double den = c->pr[i].fnorm > 0 ? c->pr[i].fnorm : 1.0;
      stats[i].iters = hs.iter;
      stats[i].rel_res = hs.rel;
      stats[i].omega_used = c->pr[i].omega;
      stats[i].t_solve_ms = ms;
      stats[i].status = r;
      stats[i].rel_rp = std::sqrt(std::max(hs.rp2, 0.0)) / den;
      stats[i].rel_ru = std::sqrt(std::max(hs.ru2, 0.0)) / den;
      stats[i].t_setup_ms = c->t_setup_ms;
      stats[i].t_omega_ms = c->t_omega_ms;
      for (int k = 0; k < PH_COUNT; ++k) stats[i].t_phase_ms[k] = tph[k];
    }
    if (r == STP_EDIVERGED) {
      worst = r;
      fail(r, "problem %d: residual diverged at iteration %d (rel %.3e)", i, hs.iter, hs.rel);
    } else if (r == STP_ENOTCONV && worst == STP_OK) {
      worst = r;
      fail(r, "problem %d: max_iter %d reached (rel %.3e)", i, c->opt.max_iter, hs.rel);
    }
  }
  return worst;
}

stp_status stp_uzawa_solve(stp_ctx* c, double* u, double* p, stp_stats* st) {
  if (!c || !u || !p) return fail(STP_EINVAL, "NULL argument (u and p are required)");
  if (c->P != 1) return fail(STP_EUNSUPPORTED, "use stp_uzawa_solve_batch for a batch context");
  return stp_uzawa_solve_batch(c, &u, &p, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

std::mutex g_tune_mu;
std::map<std::string, Schedule> g_tune_cache;

std::string tune_key(stp_ctx* c) {
  char b[96];
  snprintf(b, sizeof(b), "p%d d%d s%d r%d", c->prec, c->dim, c->spatial, c->rm);
  std::string k = b;
  for (auto& q : c->pr) {
    snprintf(b, sizeof(b), "|%d,%d,%d", q.n, q.N, q.R);
    k += b;
  }
  return k;
}

// slabs per block that knob k with exponent e gives each job (empty: knob unused)
std::vector<int> knob_sbs(stp_ctx* c, int k, int e) {
  std::vector<int> v;
  if (c->disc == STP_DISC_FEM) return v;   // finite elements: one thread per node, no tile schedule
  for (auto& q : c->pr) {
    const bool mg = c->spatial == STP_SPATIAL_MG;
    long tiles = -1;
    if (k == KN_FUSE) {
      if (c->spatial == STP_SPATIAL_MG) v.push_back(fuse_threads(e));
      continue;
    }
    if (k == KN_R0 || k == KN_R1) tiles = q.resid_tiles;
    else if (k == KN_MID) tiles = tiles_mid_d(q.dim, q.n);
    else if (k == KN_UPA0) {
      tiles = (mg && q.fuse_top > 0) ? tiles_up_d(q.dim, q.n) : -1;
      const VCycle& v = c->sites.vc[VC_A];   // register-pencil sites have a fixed shape
      if (v.up.empty() || v.up[0].jobs.empty()) tiles = -1;
    }
    else if (k < KN_UP0) {
      const int l = k - KN_DOWN0;
      tiles = (mg && l < q.fuse_top) ? tiles_down_d(q.dim, q.lv[l + 1].n) : -1;
      // the knob sets the slabs per block of the tiled down-sweeps of level l;
      // register-pencil sites have a fixed shape
      auto tiled = [&](const VCycle& v) { return size_t(l) < v.down.size() && !v.down[l].jobs.empty(); };
      if (!tiled(c->sites.vc[VC_A]) && !tiled(c->sites.vc[VC_H1])) tiles = -1;
    } else {
      const int l = k - KN_UP0;
      tiles = (mg && l < q.fuse_top) ? tiles_up_d(q.dim, q.lv[l].n) : -1;
      auto tiled = [&](const VCycle& v) { return size_t(l) < v.up.size() && !v.up[l].jobs.empty(); };
      if (!tiled(c->sites.vc[VC_A]) && !tiled(c->sites.vc[VC_H1])) tiles = -1;
    }
    if (tiles > 0) v.push_back(sched_sb(tiles, q.N, e));
  }
  return v;
}

stp_status rebuild(stp_ctx* c, const std::vector<double*>& u, const std::vector<double*>& p) {
  build_sites(c, u, p);
  if (tables_bytes(c->sites) > c->tables_bytes) return fail(STP_EDEVICE, "launch tables outgrew their reservation");
  if (!sites_fit(c)) return fail(STP_EUNSUPPORTED, "a launch exceeds the dispatch size limit");
  carve_tables(c->sites, (char*)c->ws + c->tables_off);
  return upload_all(c);
}

template <typename F>
stp_status time_ms(stp_ctx* c, int reps, F&& f, double& ms) {
  stp_status s = f();   // warm-up
  if (s != STP_OK) return s;
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  for (int r = 0; r < reps; ++r)
    if ((s = f()) != STP_OK) return s;
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  HIP_TRY(hipEventSynchronize(c->ev1));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, c->ev0, c->ev1));
  ms = double(t) / reps;
  return STP_OK;
}

void describe_schedule(stp_ctx* c) {
  std::string t;
  char b[128];
  auto knob_name = [](int k) -> std::string {
    char nb[32];
    if (k == KN_R0) return "resid_a1";
    if (k == KN_R1) return "resid_a3";
    if (k == KN_MID) return "apply_mid";
    if (k == KN_UPA0) return "up_add64_L0";
    if (k == KN_FUSE) return "fused_threads";
    if (k < KN_UP0) snprintf(nb, sizeof(nb), "down_L%d", k - KN_DOWN0);
    else snprintf(nb, sizeof(nb), "up_L%d", k - KN_UP0);
    return nb;
  };
  for (int k = 0; k < KN_COUNT; ++k) {
    std::vector<int> v = knob_sbs(c, k, c->sched.e[k]);
    if (v.empty()) continue;
    snprintf(b, sizeof(b), "%s%s:e=%d,%s=%d", t.empty() ? "" : " ", knob_name(k).c_str(), c->sched.e[k],
             k == KN_FUSE ? "threads" : "sb", v[0]);
    t += b;
    if (v.size() > 1) t += "..";
  }
  for (auto& s : c->sites.a4) {
    const char* nm = s.path == TP_FFT2 ? "fft2"
                     : s.path == TP_STOCKHAM ? "stockham"
                     : s.path == TP_BLUESTEIN ? "bluestein"
                     : s.path == TP_FOUR ? "fourstep" : "dense";
    if (s.key >= kBlueKey) snprintf(b, sizeof(b), " dst_M%d:%s", s.key - kBlueKey, nm);
    else if (s.key > 0) snprintf(b, sizeof(b), " dst_N%d:%s", s.key, nm);
    else snprintf(b, sizeof(b), " dst_other:%s", nm);
    t += b;
    if (s.path == TP_STOCKHAM || s.path == TP_BLUESTEIN || s.path == TP_FOUR) {
      snprintf(b, sizeof(b), ",C=%d", s.C);
      t += b;
    }
  }
  c->sched_text = t;
}

}  // namespace

extern "C" {

const char* stp_schedule_string(stp_ctx* c) {
  if (!c) return "";
  describe_schedule(c);
  return c->sched_text.c_str();
}

stp_status stp_autotune(stp_ctx* c, int reps, int use_cache, stp_tune_report* rep) {
  if (!c) return fail(STP_EINVAL, "NULL context");
  if (c->spatial == STP_SPATIAL_NONE) return fail(STP_EUNSUPPORTED, "context created without a spatial solver");
  reps = std::max(1, std::min(reps, 100));
  stp_tune_report r{};
  const std::string key = tune_key(c);
  stp_status s;
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c->sched = it->second;
      r.from_cache = 1;
    }
  }
  for (hipGraphExec_t* g : {&c->gexec, &c->gexecA, &c->gexecH})
    if (*g) {   // the launch shapes change: capture again at the next solve
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  const size_t P = c->pr.size();
  std::vector<double*> nul(P, nullptr);
  if (r.from_cache) {
    if ((s = rebuild(c, nul, nul)) != STP_OK) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (rep) *rep = r;
    return STP_OK;
  }
  // scratch iterates: the tuner runs real launches on the context's buffers
  size_t total = 0;
  for (auto& q : c->pr) total += size_t(2) * q.N * q.g0.npts;
  double* tmp = nullptr;
  bool owned = false;
  if ((s = scratch_get(c, total, &tmp, &owned)) != STP_OK) return s;
  std::vector<double*> tu(P), tp(P);
  {
    size_t off = 0;
    for (size_t i = 0; i < P; ++i) {
      const size_t nv = size_t(c->pr[i].N) * c->pr[i].g0.npts;
      tu[i] = tmp + off;
      tp[i] = tmp + off + nv;
      off += 2 * nv;
    }
  }
  const stp_options saved = c->opt;
  const bool kt_saved = c->kt.on;
  c->opt.tol = 0.0;                 // no stop test while tuning
  c->opt.max_iter = 1 << 30;
  c->kt.on = false;
  auto body = [&]() -> stp_status {
    HIP_TRY(hipMemsetAsync(tmp, 0, total * 8, c->stream));
    for (size_t i = 0; i < P; ++i) {
      c->state_host[i] = DevState{};
      c->state_host[i].fnorm = c->pr[i].fnorm;
      HIP_TRY(hipMemcpyAsync(c->pr[i].state, &c->state_host[i], sizeof(DevState), hipMemcpyHostToDevice, c->stream));
    }
    stp_status st;
    if ((st = rebuild(c, tu, tp)) != STP_OK) return st;
    auto iter = [&]() { return c->impl->iteration(); };
    if ((st = iter()) != STP_OK) return st;
    if ((st = time_ms(c, reps, iter, r.iter_ms_before)) != STP_OK) return st;
    // tile launches: slabs per block, knob by knob
    for (int k = 0; k < KN_COUNT; ++k) {
      const std::vector<int> base = knob_sbs(c, k, 0);
      if (base.empty()) continue;
      ++r.knobs_tuned;
      std::vector<std::vector<int>> seen(1, base);
      double best_t = 0;
      if ((st = time_ms(c, reps, [&]() { return c->impl->launch_knob(k); }, best_t)) != STP_OK) return st;
      ++r.candidates;
      int best_e = 0;
      for (int e = -3; e <= 3; ++e) {
        if (e == 0) continue;
        const std::vector<int> v = knob_sbs(c, k, e);
        if (std::find(seen.begin(), seen.end(), v) != seen.end()) continue;
        seen.push_back(v);
        c->sched.e[k] = e;
        if ((st = rebuild(c, tu, tp)) != STP_OK) {
          c->sched.e[k] = best_e;
          if (st == STP_EUNSUPPORTED) continue;
          return st;
        }
        double t = 0;
        if ((st = time_ms(c, reps, [&]() { return c->impl->launch_knob(k); }, t)) != STP_OK) return st;
        ++r.candidates;
        if (t < 0.98 * best_t) {   // keep the heuristic unless a choice is clearly faster
          best_t = t;
          best_e = e;
        }
      }
      c->sched.e[k] = best_e;
      if ((st = rebuild(c, tu, tp)) != STP_OK) return st;
    }
    // time transforms: path and Stockham columns per power-of-two step count
    const size_t tcb = tc_bytes(c->prec);
    for (size_t g = 0; g < c->sites.a4.size(); ++g) {
      const int key = c->sites.a4[g].key;
      if (key <= 0) continue;
      std::vector<TransformChoice> cand;
      if (key >= kBlueKey) {   // Bluestein group of FFT length M (every N of the group <= M / 2)
        const int M = key - kBlueKey;
        for (int C = 1; C <= 16; C *= 2)
          if (M * C <= 4096 && bluestein_lds(M, C, tcb) <= kMaxLds) cand.push_back({TP_BLUESTEIN, C});
        if (M <= 128) cand.push_back({TP_DENSE, 0});
      } else {
        const int N = key;
        if (N >= 4 && N <= 256) cand.push_back({TP_FFT2, 0});
        for (int C = 1; C <= 16; C *= 2)
          if (N * C <= 4096 && stockham_lds(N, C, tcb) <= kMaxLds) cand.push_back({TP_STOCKHAM, C});
        if (four_step_n(N, tcb))
          for (int C = 1; C <= 16; C *= 2)
            if (four_n1(N) * C <= 4096 && four_lds(N, C, tcb) <= kMaxLds) cand.push_back({TP_FOUR, C});
        if (N <= 64) cand.push_back({TP_DENSE, 0});
      }
      const Site<TimeJob> cur = c->sites.a4[g];
      TransformChoice best{cur.path, cur.C};
      double best_t = 0;
      if ((st = time_ms(c, reps, [&]() { return c->impl->launch_transform(int(g)); }, best_t)) != STP_OK) return st;
      ++r.knobs_tuned;
      ++r.candidates;
      for (const auto& ch : cand) {
        if (ch.path == best.path && ch.C == best.C) continue;
        c->sched.tpath[key] = ch;
        if ((st = rebuild(c, tu, tp)) != STP_OK) {
          c->sched.tpath[key] = best;
          if (st == STP_EUNSUPPORTED) continue;
          return st;
        }
        double t = 0;
        if ((st = time_ms(c, reps, [&]() { return c->impl->launch_transform(int(g)); }, t)) != STP_OK) return st;
        ++r.candidates;
        if (t < 0.98 * best_t) {
          best_t = t;
          best = ch;
        }
      }
      c->sched.tpath[key] = best;
      if ((st = rebuild(c, tu, tp)) != STP_OK) return st;
    }
    return time_ms(c, reps, iter, r.iter_ms_after);
  };
  s = body();
  c->opt = saved;
  c->kt.on = kt_saved;
  const stp_status s2 = rebuild(c, nul, nul);   // tables as after stp_create: u, p bound at the next solve
  scratch_put(c, tmp, owned);
  if (s != STP_OK) return s;
  if (s2 != STP_OK) return s2;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = c->sched;
  }
  if (rep) *rep = r;
  return STP_OK;
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

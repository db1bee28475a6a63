// Host runtime behind the C ABI (include/lddmm.h): argument checks, pyramid
// geometry, workspace layout, and the launch sequence of the descent.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <list>
#include <vector>

#include "internal.h"
#include "lddmm.h"
#include "lddmm_cnn.h"

namespace lddmm {

// ------------------------------------------------------------ profiling ----
// Events bracket each launch of an enabled class on its own stream.
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  long long vox;
};
static unsigned g_prof_mask = 0;
static long long g_prof_min_vox = 0;
static std::vector<ProfRec> g_prof_rec;
static std::vector<hipEvent_t> g_prof_pool;
static size_t g_prof_used = 0;

static hipEvent_t prof_event() {
  if (g_prof_used == g_prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof_pool.push_back(e);
  }
  return g_prof_pool[g_prof_used++];
}

void prof_open(int cls, long long vox, hipStream_t s, hipEvent_t* a) {
  *a = nullptr;
  if ((g_prof_mask & (1u << cls)) && vox >= g_prof_min_vox) {
    *a = prof_event();
    if (*a) hipEventRecord(*a, s);
  }
}

void prof_close(int cls, long long vox, hipStream_t s, hipEvent_t a) {
  if (!a) return;
  hipEvent_t b = prof_event();
  if (!b) return;
  hipEventRecord(b, s);
  g_prof_rec.push_back({cls, a, b, vox});
}

static bool is_7smooth(int n) {
  for (int p : {2, 3, 5, 7})
    while (n > 1 && n % p == 0) n /= p;
  return n == 1;
}

static int smooth7(int n) {
  int m = n < 2 ? 2 : n;
  while (!is_7smooth(m)) ++m;
  return m;
}

struct Level {
  Geom g;
  int N[3];          // user grid of this level (x, y, z)
  FFTPlan px, py, pz;
};

static Geom make_geom(int nx, int ny, int nz, double h) {
  Geom g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.hx = nx / 2 + 1;
  g.hs = (g.hx + 15) / 16 * 16;
  g.n = (long long)nx * ny * nz;
  g.nspec = (long long)g.hs * ny * nz;
  g.h = (float)h;
  g.inv_h = (float)(1.0 / h);
  g.fx = make_fastdiv((uint32_t)nx);
  g.fy = make_fastdiv((uint32_t)ny);
  g.fz = make_fastdiv((uint32_t)nz);
  g.fhx = make_fastdiv((uint32_t)g.hx);
  return g;
}

// Levels coarsest first; the coarsest computational grid is 7-smooth and each
// finer one doubles it, so all levels nest.
static bool build_levels(const lddmm_grid* grid, int L, Level* lv) {
  const int N[3] = {grid->nx, grid->ny, grid->nz};
  const int f = 1 << (L - 1);
  int Pc[3];
  for (int d = 0; d < 3; ++d) Pc[d] = smooth7((N[d] + f - 1) / f);
  for (int li = 0; li < L; ++li) {
    const int lev = L - 1 - li;        // 0 = finest
    const int s = 1 << lev;
    int P[3];
    for (int d = 0; d < 3; ++d) {
      P[d] = Pc[d] * (f / s);
      lv[li].N[d] = (N[d] + s - 1) / s;
      if (P[d] < 2 || P[d] > LDDMM_MAX_DIM) return false;
    }
    lv[li].g = make_geom(P[0], P[1], P[2], grid->spacing * (double)s);
    if (!make_plan(P[0], &lv[li].px) || !make_plan(P[1], &lv[li].py) ||
        !make_plan(P[2], &lv[li].pz))
      return false;
  }
  return true;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state, partR, partD, partI, partDet, trace, tw[3], lam[3];
  size_t J0, J1, v0, v1, u0, u1, J0t, r, b, S, ub, misc, ptab, total;
  size_t bT, ST, ttab;             // time-batched K: T body forces, spectra, tables (0: none)
  size_t Joff[LDDMM_MAX_LEVELS];   // per-level offsets (floats) inside J0 / J1
  int n_u0;                         // u0 slots
};

struct Config {
  int L, T, C, nch, ch[2];
  float w[2];
  int img_ch, img_weighted, img_slot;
  Level lv[LDDMM_MAX_LEVELS];
  int rows;
  int ck;            // exact gradient: checkpoint spacing (0 = keep every u0_j)
  int rk4;           // departure points by fourth-order Runge-Kutta (LDDMM_FLAG_RK4)
  int kt_mask;       // bit li: level li of a descent smooths its T body forces in one batch
};

// Levels of a descent whose K passes run over all T time steps at once: up to
// this many voxels a level's passes are short and bound by the latency of one
// block's phases (a 140 x 80 x 120 pass has 360 blocks for 256 CUs), and ten
// times the blocks fill the chip.  The finest atlas level (10.75 M voxels)
// fills it alone.
constexpr long long kTimeBatchMaxVoxels = 1LL << 21;
static int g_k_time_batch = 1;

static void set_k_time_batch(int on) { g_k_time_batch = on ? 1 : 0; }

// u0 storage of the exact gradient.  Without recompute slot j holds u0_j.  With
// checkpoints every ck steps: slots [0, nck) hold u0 at j = 0, ck, 2 ck, ... and
// T; the next max(2, ck - 1) slots are scratch (ping-pong during the full
// forward sweep, then the interior steps of the segment being recomputed).
struct U0Plan {
  int ck, nck, nslots;
};

static U0Plan u0_plan(int T, int ck) {
  U0Plan p{};
  p.ck = ck;
  if (ck <= 0 || ck >= T) {
    p.ck = 0;
    p.nck = T + 1;
    p.nslots = T + 1;
    return p;
  }
  p.nck = (T + ck - 1) / ck + 1;
  p.nslots = p.nck + (ck - 1 > 2 ? ck - 1 : 2);
  return p;
}

// Slot of a checkpoint step (j multiple of ck, or T).
static int ck_slot(const U0Plan& p, int j, int T) {
  if (p.ck == 0) return j;
  return j == T ? p.nck - 1 : j / p.ck;
}
static bool is_ck(const U0Plan& p, int j, int T) { return p.ck == 0 || j == T || j % p.ck == 0; }

static int trace_rows(const lddmm_params* p) {
  int rows = 0;
  for (int l = 0; l < p->n_levels; ++l) rows += p->iters[l] + 1;
  return rows;
}

static int check_params(const lddmm_grid* grid, const lddmm_params* p, int multilevel) {
  if (!grid || !p) return LDDMM_EINVAL;
  if (grid->nx < 2 || grid->ny < 2 || grid->nz < 2) return LDDMM_EINVAL;
  if (grid->nx > LDDMM_MAX_DIM || grid->ny > LDDMM_MAX_DIM || grid->nz > LDDMM_MAX_DIM)
    return LDDMM_EINVAL;
  if (!(grid->spacing > 0.0) || !std::isfinite(grid->spacing)) return LDDMM_EINVAL;
  if ((long long)grid->nx * grid->ny * grid->nz >= (1LL << 29)) return LDDMM_EINVAL;
  if (!(p->alpha >= 0.0) || !(p->gamma > 0.0) || !(p->sigma > 0.0)) return LDDMM_EINVAL;
  if (!std::isfinite(p->alpha) || !std::isfinite(p->gamma) || !std::isfinite(p->sigma))
    return LDDMM_EINVAL;
  if (p->n_timesteps < 1 || p->n_timesteps > LDDMM_MAX_T) return LDDMM_EINVAL;
  if (multilevel) {
    if (p->n_levels < 1 || p->n_levels > LDDMM_MAX_LEVELS) return LDDMM_EINVAL;
    for (int l = 0; l < p->n_levels; ++l)
      if (p->iters[l] < 0 || p->iters[l] > 1000000) return LDDMM_EINVAL;
    if (!(p->step > 0.0) || !std::isfinite(p->step)) return LDDMM_EINVAL;
  }
  if (!(p->weight[0] >= 0.0) || !(p->weight[1] >= 0.0)) return LDDMM_EINVAL;
  return LDDMM_OK;
}

static int make_config(const lddmm_grid* grid, const lddmm_params* p, int has_img, int multilevel,
                       Config* c) {
  int rc = check_params(grid, p, multilevel);
  if (rc) return rc;
  c->L = multilevel ? p->n_levels : 1;
  c->T = p->n_timesteps;
  c->C = has_img ? 2 : 1;
  c->nch = 0;
  for (int k = 0; k < c->C; ++k) {
    if (p->weight[k] > 0.0) {
      c->ch[c->nch] = k;
      c->w[c->nch] = (float)p->weight[k];
      ++c->nch;
    }
  }
  if (c->nch == 0) return LDDMM_EINVAL;
  c->img_ch = has_img ? 1 : -1;
  c->img_weighted = 0;
  c->img_slot = 0;
  for (int k = 0; k < c->nch; ++k)
    if (c->ch[k] == 1) {
      c->img_weighted = 1;
      c->img_slot = k;
    }
  if (!build_levels(grid, c->L, c->lv)) return LDDMM_EINVAL;
  c->rows = multilevel ? trace_rows(p) : 1;
  c->rk4 = (p->flags & LDDMM_FLAG_RK4) ? 1 : 0;
  c->ck = (p->flags & LDDMM_FLAG_RECOMPUTE_PHI) ? (p->checkpoint_every > 0 ? p->checkpoint_every
                                                                            : 1)
                                                : 0;
  c->kt_mask = 0;
  if (multilevel)
    for (int l = 0; l < c->L; ++l)
      if (c->lv[l].g.n <= kTimeBatchMaxVoxels) c->kt_mask |= 1 << l;
  return LDDMM_OK;
}

static Layout make_layout(const Config& c) {
  Layout o{};
  const Geom& gf = c.lv[c.L - 1].g;
  const size_t n = (size_t)gf.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off);
    const size_t at = off;
    off += bytes;
    return at;
  };
  o.state = take(sizeof(State));
  o.partR = take(sizeof(double) * kPartMax * c.T);
  o.partD = take(sizeof(double) * kPartMax);
  o.partI = take(sizeof(double) * kPartMax);
  o.partDet = take(sizeof(double) * kPartMax * c.T);
  o.trace = take(sizeof(double) * 8 * (size_t)(c.rows > 0 ? c.rows : 1));
  const int P[3] = {gf.nx, gf.ny, gf.nz};
  for (int d = 0; d < 3; ++d) o.tw[d] = take(sizeof(float2) * P[d]);
  for (int d = 0; d < 3; ++d) o.lam[d] = take(sizeof(double) * P[d]);
  size_t jt = 0;
  for (int l = 0; l < c.L; ++l) {
    o.Joff[l] = jt;
    jt += (size_t)c.C * c.lv[l].g.n;
  }
  o.J0 = take(sizeof(float) * jt);
  o.J1 = take(sizeof(float) * jt);
  o.v0 = take(sizeof(float) * 3 * n * c.T);
  o.v1 = take(sizeof(float) * 3 * n * c.T);
  o.n_u0 = u0_plan(c.T, c.ck).nslots;
  o.u0 = take(sizeof(float) * 3 * n * o.n_u0);
  o.u1 = take(sizeof(float) * 3 * n * 2);
  o.J0t = take(sizeof(float) * n * c.nch * c.T);
  o.r = take(sizeof(float) * n * c.nch);
  o.b = take(sizeof(float) * 3 * n);
  o.S = take(sizeof(float2) * 3 * (size_t)gf.nspec);
  o.ub = take(sizeof(float) * 3 * n * 2);
  o.misc = take(sizeof(int) * 64);
  o.ptab = take(sizeof(PairTab));
  o.bT = o.ST = o.ttab = 0;
  if (c.kt_mask) {
    size_t nmax = 0, smax = 0;
    for (int l = 0; l < c.L; ++l)
      if ((c.kt_mask >> l) & 1) {
        nmax = std::max(nmax, (size_t)c.lv[l].g.n);
        smax = std::max(smax, (size_t)c.lv[l].g.nspec);
      }
    o.bT = take(sizeof(float) * 3 * nmax * c.T);
    o.ST = take(sizeof(float2) * 3 * smax * c.T);
    o.ttab = take(sizeof(PairTab) * c.T);
  }
  o.total = align_up(off);
  return o;
}

// Device pointers of one problem's workspace at one level.
struct Ctx {
  Config cfg;
  Layout lay;
  char* ws;
  State* st;
  double *partR, *partD, *partI, *partDet, *trace;
  float2* tw[3];
  double* lam[3];
  float *J0, *J1, *v[2], *u0, *u1, *J0t, *r, *b, *ub;
  int* misc;
  PairTab* ptab;
  float2* S;
  double alpha, gamma, sigma;
  int guard;
  // time-batched K (levels in cfg.kt_mask): body forces [T][3][n], spectra
  // [T][3][nspec], one device table per time step, and the host copies behind
  // them (one set per table build, kept until the call returns, so that no
  // copy still in flight reads a buffer that is being rewritten)
  float* bT;
  float2* ST;
  PairTab* ttab;
  std::list<std::vector<PairTab>> htab;
  int ttab_level;
  UpdArgs ttab_upd;
};

static void bind(Ctx& c, void* ws) {
  c.ws = (char*)ws;
  const Layout& o = c.lay;
  c.st = (State*)(c.ws + o.state);
  c.partR = (double*)(c.ws + o.partR);
  c.partD = (double*)(c.ws + o.partD);
  c.partI = (double*)(c.ws + o.partI);
  c.partDet = (double*)(c.ws + o.partDet);
  c.trace = (double*)(c.ws + o.trace);
  for (int d = 0; d < 3; ++d) {
    c.tw[d] = (float2*)(c.ws + o.tw[d]);
    c.lam[d] = (double*)(c.ws + o.lam[d]);
  }
  c.J0 = (float*)(c.ws + o.J0);
  c.J1 = (float*)(c.ws + o.J1);
  c.v[0] = (float*)(c.ws + o.v0);
  c.v[1] = (float*)(c.ws + o.v1);
  c.u0 = (float*)(c.ws + o.u0);
  c.u1 = (float*)(c.ws + o.u1);
  c.J0t = (float*)(c.ws + o.J0t);
  c.r = (float*)(c.ws + o.r);
  c.b = (float*)(c.ws + o.b);
  c.S = (float2*)(c.ws + o.S);
  c.ub = (float*)(c.ws + o.ub);
  c.misc = (int*)(c.ws + o.misc);
  c.ptab = (PairTab*)(c.ws + o.ptab);
  c.bT = o.bT ? (float*)(c.ws + o.bT) : nullptr;
  c.ST = o.ST ? (float2*)(c.ws + o.ST) : nullptr;
  c.ttab = o.ttab ? (PairTab*)(c.ws + o.ttab) : nullptr;
  c.ttab_level = -1;
}

static void level_tables(Ctx& c, const Level& L, hipStream_t s) {
  const int P[3] = {L.g.nx, L.g.ny, L.g.nz};
  for (int d = 0; d < 3; ++d) {
    launch_twiddles(c.tw[d], P[d], s);
    launch_lambda(c.lam[d], P[d], (double)L.g.h, s);
  }
}

// Forward sweep of the velocity selected by st->eval (vA/vB) for steps
// j in [j_beg, j_end): reads u0_j from slot sl[j], writes u0_{j+1} to slot sl[j+1],
// plus deformed templates, r and the energy partials.
static void forward_steps(Ctx& c, int li, const float* vA, const float* vB, const int* sl, int j_beg,
                          int j_end, hipStream_t s) {
  const Config& k = c.cfg;
  const Level& L = k.lv[li];
  const long long n = L.g.n;
  for (int j = j_beg; j < j_end; ++j) {
    FwdArgs a{};
    a.g = L.g;
    a.vA = vA;
    a.vB = vB;
    a.j = j;
    a.T = k.T;
    a.dt = 1.0f / (float)k.T;
    a.alpha = (float)c.alpha;
    a.gamma = (float)c.gamma;
    a.u_cur = c.u0 + (long long)sl[j] * 3 * n;
    a.u_next = c.u0 + (long long)sl[j + 1] * 3 * n;
    a.J0 = c.J0 + c.lay.Joff[li];
    a.J1 = c.J1 + c.lay.Joff[li];
    a.nch = k.nch;
    a.ch[0] = k.ch[0];
    a.ch[1] = k.nch > 1 ? k.ch[1] : k.ch[0];
    a.w[0] = k.w[0];
    a.w[1] = k.nch > 1 ? k.w[1] : 0.f;
    a.img_ch = k.img_ch;
    a.img_weighted = k.img_weighted;
    a.img_slot = k.img_slot;
    a.J0t_next = c.J0t + (long long)(j + 1 < k.T ? j + 1 : 0) * k.nch * n;
    a.r = c.r;
    a.partR = c.partR + (long long)j * kPartMax;
    a.partD = c.partD;
    a.partI = c.partI;
    a.st = c.st;
    a.rk4 = k.rk4;
    a.zmarch = forward_zmarch(L.g);
    a.staged = forward_staged(L.g);
    ProfScope ps((j == 0 || j == k.T - 1) ? LDDMM_PROF_FORWARD_EDGE : LDDMM_PROF_FORWARD, n, s);
    launch_forward(a, s);
  }
}

static void forward_sweep(Ctx& c, int li, const float* vA, const float* vB, bool keep_all,
                          hipStream_t s) {
  int sl[LDDMM_MAX_T + 1];
  for (int j = 0; j <= c.cfg.T; ++j) sl[j] = keep_all ? j : (j & 1);
  forward_steps(c, li, vA, vB, sl, 0, c.cfg.T, s);
}

static float* u0_final(Ctx& c, int li, bool keep_all) {
  const long long n = c.cfg.lv[li].g.n;
  const int T = c.cfg.T;
  return c.u0 + (long long)(keep_all ? T : (T & 1)) * 3 * n;
}

// FFT pass parameters of one problem at one level.
static FftPair make_fft(Ctx& c, int li, int need_mode, FftLaunch* L) {
  FftPair f{};
  const Level& lv = c.cfg.lv[li];
  f.g = lv.g;
  f.px = lv.px;
  f.py = lv.py;
  f.pz = lv.pz;
  for (int d = 0; d < 3; ++d) {
    f.tw[d] = c.tw[d];
    f.lam[d] = c.lam[d];
  }
  f.alpha = c.alpha;
  f.gamma = c.gamma;
  f.b = c.b;
  f.S = c.S;
  f.st = c.st;
  f.need_mode = need_mode;
  fft_tiles(f, L);
  return f;
}

// K smoothing of c.b followed by the x-inverse epilogue.
static void smooth_and_update(Ctx& c, int li, const UpdArgs& u, int need_mode, hipStream_t s) {
  const long long n = c.cfg.lv[li].g.n;
  FftLaunch L;
  const FftPair f = make_fft(c, li, need_mode, &L);
  {
    ProfScope ps(LDDMM_PROF_FFT_X, n, s);
    launch_fft_x_fwd(f, L, s);
  }
  if (!f.fused) {
    ProfScope ps(LDDMM_PROF_FFT_Y, n, s);
    launch_fft_y(f, L, 0, s);
  }
  {
    ProfScope ps(LDDMM_PROF_FFT_ZK, n, s);
    launch_fft_z_K(f, L, s);
  }
  if (!f.fused) {
    ProfScope ps(LDDMM_PROF_FFT_YINV, n, s);
    launch_fft_y(f, L, 1, s);
  }
  {
    ProfScope ps(LDDMM_PROF_FFT_XINV, n, s);
    launch_fft_x_inv(f, L, u, s);
  }
}

// K b_j and the epilogue of every time step j at once, from the body forces
// b_j in c.bT: the batched passes with one table per time step (its FftPair on
// b_j and the j-th slice of c.ST, its epilogue in upd[0]).  The per-line
// arithmetic is that of the single-step launches, so the results are the same
// bits.  The tables are written once per level and epilogue.
static void smooth_and_update_all(Ctx& c, int li, const UpdArgs& u, int need_mode,
                                  hipStream_t s) {
  const Config& k = c.cfg;
  const long long n = k.lv[li].g.n;
  FftLaunch L;
  const FftPair f = make_fft(c, li, need_mode, &L);
  const UpdArgs& t = c.ttab_upd;
  if (c.ttab_level != li || t.kind != u.kind || t.vA != u.vA || t.vB != u.vB ||
      t.vfix != u.vfix || t.out != u.out || t.need_mode != u.need_mode) {
    std::vector<PairTab>& ht = c.htab.emplace_back(k.T, PairTab{});
    for (int j = 0; j < k.T; ++j) {
      PairTab& h = ht[j];
      h.fft = f;
      h.fft.b = c.bT + (long long)j * 3 * n;
      h.fft.S = c.ST + (long long)j * 3 * f.g.nspec;
      h.upd[0] = u;
      h.upd[0].j = j;
    }
    hipMemcpyAsync(c.ttab, ht.data(), sizeof(PairTab) * k.T, hipMemcpyHostToDevice, s);
    c.ttab_level = li;
    c.ttab_upd = u;
  }
  for (int j0 = 0; j0 < k.T; j0 += kMaxBatch) {
    const int np = std::min(kMaxBatch, k.T - j0);
    BatchRef bx{}, by{}, bz{};
    bx.np = by.np = bz.np = np;
    for (int p = 0; p <= np; ++p) {
      bx.off[p] = p * L.x_tiles;
      by.off[p] = p * L.y_tiles;
      bz.off[p] = p * L.z_tiles;
    }
    for (int p = 0; p < np; ++p) bx.tab[p] = by.tab[p] = bz.tab[p] = c.ttab + j0 + p;
    // fused x + y passes with the single-problem launch's block size
    {
      ProfScope ps(LDDMM_PROF_FFT_X, n, s);
      if (!(f.fused && launch_fft_fused_batched(0, bx, f.g, L.x_lds, 0, s)))
        launch_fft_batched(0, bx, L.ex, L.x_lds, 0, s);
    }
    if (!f.fused) {
      ProfScope ps(LDDMM_PROF_FFT_Y, n, s);
      launch_fft_batched(1, by, L.ey, L.y_lds, 0, s);
    }
    {
      ProfScope ps(LDDMM_PROF_FFT_ZK, n, s);
      launch_fft_batched(2, bz, L.ez, L.z_lds, 0, s);
    }
    if (!f.fused) {
      ProfScope ps(LDDMM_PROF_FFT_YINV, n, s);
      launch_fft_batched(3, by, L.ey, L.y_lds, 0, s);
    }
    {
      ProfScope ps(LDDMM_PROF_FFT_XINV, n, s);
      if (!(f.fused && launch_fft_fused_batched(1, bx, f.g, L.x_lds, 0, s)))
        launch_fft_batched(4, bx, L.ex, L.x_lds, 0, s);
    }
  }
}

// Backward sweep: maps u1_j, body forces b_j, K b_j and the epilogue per j.
// With with_grad = false only the maps are computed (u1_0 ends in slot 0).
// With time_batch, every b_j goes to its own slice of c.bT and K and the
// epilogue of all time steps follow the sweep (the sweep reads the iterate
// that the epilogue does not write, so the order changes nothing).
static void backward_sweep(Ctx& c, int li, float* vA, float* vB, const float* vfix, bool with_grad,
                           int upd_kind, float* gout, int need_mode, hipStream_t s,
                           bool smooth = true, bool time_batch = false) {
  const Config& k = c.cfg;
  const Level& L = k.lv[li];
  const long long n = L.g.n;
  time_batch = time_batch && with_grad && smooth && c.bT != nullptr && ((k.kt_mask >> li) & 1);
  for (int j = k.T - 1; j >= (with_grad ? -1 : 0); --j) {
    BwdArgs a{};
    a.g = L.g;
    a.vA = vA;
    a.vB = vB;
    a.vfix = vfix;
    a.T = k.T;
    a.dt = 1.0f / (float)k.T;
    a.j = j;
    a.u_next = (j == k.T - 1) ? nullptr : c.u1 + (long long)((j + 1) & 1) * 3 * n;
    a.u_cur = j >= 0 ? c.u1 + (long long)(j & 1) * 3 * n : nullptr;
    const int jb = j + 1;
    a.jb = (with_grad && jb <= k.T - 1) ? jb : -1;
    if (a.jb == 0) {
      a.J0t = c.J0 + c.lay.Joff[li] + (long long)k.ch[0] * n;
      a.cstride = k.nch > 1 ? (long long)(k.ch[1] - k.ch[0]) * n : n;
    } else {
      a.J0t = c.J0t + (long long)jb * k.nch * n;
      a.cstride = n;
    }
    a.r = c.r;
    a.nch = k.nch;
    a.w[0] = k.w[0];
    a.w[1] = k.nch > 1 ? k.w[1] : 0.f;
    a.coef = (float)(2.0 / (c.sigma * c.sigma));
    a.b = (time_batch && a.jb >= 0) ? c.bT + (long long)a.jb * 3 * n : c.b;
    a.partDet = c.partDet + (long long)(a.jb >= 0 ? a.jb : 0) * kPartMax;
    a.st = c.st;
    a.need_mode = need_mode;
    a.rk4 = k.rk4;
    // the same choice as backward_partials(), which sizes the min-det reduction
    a.staged = backward_staged(L.g);
    if (a.j < 0 && a.jb < 0) continue;
    {
      const bool both = a.j >= 0 && a.u_next != nullptr && a.jb >= 0;
      ProfScope ps(both ? LDDMM_PROF_BACKWARD : LDDMM_PROF_BACKWARD_EDGE, n, s);
      launch_backward(a, s);
    }
    if (a.jb >= 0 && smooth && !time_batch) {
      UpdArgs u{};
      u.kind = upd_kind;
      u.j = a.jb;
      u.vA = vA;
      u.vB = vB;
      u.vfix = vfix;
      u.out = gout;
      u.st = c.st;
      u.need_mode = need_mode;
      smooth_and_update(c, li, u, need_mode, s);
    }
  }
  if (time_batch) {
    UpdArgs u{};
    u.kind = upd_kind;
    u.vA = vA;
    u.vB = vB;
    u.vfix = vfix;
    u.out = gout;
    u.st = c.st;
    u.need_mode = need_mode;
    smooth_and_update_all(c, li, u, need_mode, s);
  }
}

static void decide(Ctx& c, int li, int init, double* trace, hipStream_t s);

// Outputs of the final iterate (buffer 0) at the finest level: phi_10 (if asked),
// phi_01 (if asked) and the min det of its maps phi_{t_j,1}, which decides
// LDDMM_WFOLD.  The forward sweep gives the deformed templates and the residual
// the body-force steps read; the body forces themselves are discarded.
static void final_outputs(Ctx& c, float* phi10, float* phi01, hipStream_t s) {
  const Config& k = c.cfg;
  const int top = k.L - 1;
  const Level& L = k.lv[top];
  forward_sweep(c, top, c.v[0], c.v[1], false, s);
  if (phi10)
    launch_crop3(u0_final(c, top, false), L.g, L.N[0], L.N[1], L.N[2], phi10, s);
  backward_sweep(c, top, c.v[0], c.v[1], c.v[0], true, UPD_STEP, nullptr, -1, s, false);
  launch_final_det(c.st, c.partDet, k.T, backward_partials(L.g), s);
  if (phi01) launch_crop3(c.u1, L.g, L.N[0], L.N[1], L.N[2], phi01, s);
}

// Exact gradient dE/dv (reverse mode) of the single-level energy at v.
static void exact_gradient(Ctx& c, const float* v, float* grad, hipStream_t s) {
  const Config& k = c.cfg;
  const Level& L = k.lv[0];
  const long long n = L.g.n;
  const int T = k.T;
  const U0Plan up = u0_plan(T, k.ck);
  // full forward sweep, keeping u0 at the checkpoints (every step without recompute)
  int sl[LDDMM_MAX_T + 1];
  int scratch = 0;
  for (int j = 0; j <= T; ++j) {
    if (is_ck(up, j, T)) {
      sl[j] = ck_slot(up, j, T);
    } else {
      sl[j] = up.nck + (scratch & 1);
      ++scratch;
    }
  }
  // u0_0 = 0 is implicit in the forward kernels; the reverse step j = 0 reads it
  launch_fill(c.u0 + (long long)sl[0] * 3 * n, 3 * n, 0.f, s);
  forward_steps(c, 0, v, v, sl, 0, T, s);
  decide(c, 0, 1, c.trace, s);
  GradArgs a{};
  a.g = L.g;
  a.nch = k.nch;
  a.J0 = c.J0;
  a.ch[0] = k.ch[0];
  a.ch[1] = k.nch > 1 ? k.ch[1] : k.ch[0];
  a.wc[0] = k.w[0];
  a.wc[1] = k.nch > 1 ? k.w[1] : 0.f;
  const double h = (double)L.g.h;
  a.coef = (float)(2.0 * h * h * h / (c.sigma * c.sigma));
  a.r = c.r;
  a.dt = 1.0f / (float)T;
  a.alpha = (float)c.alpha;
  a.gamma = (float)c.gamma;
  a.reg = (float)(2.0 / T * h * h * h);
  a.w = c.b;
  a.radius = c.misc;
  a.overflow = c.misc + 1;
  a.u = c.u0 + (long long)sl[T] * 3 * n;
  a.ub_out = c.ub + (long long)(T & 1) * 3 * n;
  launch_ubar_init(a, s);
  int seg_lo = -1;   // first step of the segment whose interior is recomputed
  for (int j = T - 1; j >= 0; --j) {
    int uslot;
    if (is_ck(up, j, T)) {
      uslot = ck_slot(up, j, T);
    } else {
      const int j0 = (j / up.ck) * up.ck;
      if (seg_lo != j0) {
        // recompute u0_{j0+1} .. u0_{j} from the checkpoint at j0 into scratch slots
        int rs[LDDMM_MAX_T + 1];
        const int j1 = (j0 + up.ck < T ? j0 + up.ck : T);
        for (int m = j0; m <= j1; ++m) rs[m] = m == j0 ? ck_slot(up, j0, T) : up.nck + (m - j0 - 1);
        forward_steps(c, 0, v, v, rs, j0, j1 - 1, s);
        seg_lo = j0;
      }
      uslot = up.nck + (j - j0 - 1);
    }
    a.u = c.u0 + (long long)uslot * 3 * n;
    a.v = v + (long long)j * 3 * n;
    a.ub_in = c.ub + (long long)((j + 1) & 1) * 3 * n;
    a.ub_out = c.ub + (long long)(j & 1) * 3 * n;
    a.grad = grad + (long long)j * 3 * n;
    launch_grad_step(a, s);
  }
}

static void decide(Ctx& c, int li, int init, double* trace, hipStream_t s) {
  const Level& L = c.cfg.lv[li];
  const int nb = forward_tiles(L.g);
  const int nbw = backward_partials(L.g);
  const double h = (double)L.g.h;
  ProfScope ps(LDDMM_PROF_OTHER, 0, s);
  launch_decide(c.st, c.partR, c.cfg.T, c.partD, c.partI, c.partDet, nb, nbw, c.cfg.C > 1,
                1.0 / c.cfg.T, h * h * h, 1.0 / (c.sigma * c.sigma), c.guard, trace, init, s);
}

// Copy the current iterate into buffer 0 (kernel reads st->base).
__global__ void k_canon(float* v0, const float* v1, long long count, const State* st) {
  if (st->base == 0) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    v0[i] = v1[i];
}

__global__ void k_set_base(State* st, int base, int mode) {
  if (threadIdx.x == 0) {
    st->base = base;
    st->eval = base;
    if (mode >= 0) st->mode = mode;
  }
}

static void canonicalize(Ctx& c, long long count, hipStream_t s) {
  long long b = (count + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_canon, dim3((unsigned)b), dim3(256), 0, s, c.v[0], c.v[1], count, c.st);
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(64), 0, s, c.st, 0, -1);
}

static void setup_images(Ctx& c, const lddmm_problem* p, hipStream_t s) {
  const Config& k = c.cfg;
  const int top = k.L - 1;
  const Geom& gf = k.lv[top].g;
  const int* N = k.lv[top].N;
  float* J0f = c.J0 + c.lay.Joff[top];
  float* J1f = c.J1 + c.lay.Joff[top];
  launch_pad(p->template_mask, N[0], N[1], N[2], J0f, gf, s);
  launch_pad(p->target_mask, N[0], N[1], N[2], J1f, gf, s);
  if (k.C > 1) {
    launch_pad(p->template_image, N[0], N[1], N[2], J0f + gf.n, gf, s);
    launch_pad(p->target_image, N[0], N[1], N[2], J1f + gf.n, gf, s);
  }
  for (int li = top - 1; li >= 0; --li) {
    launch_down2(c.J0 + c.lay.Joff[li + 1], k.lv[li + 1].g, c.J0 + c.lay.Joff[li], k.lv[li].g, k.C,
                 s);
    launch_down2(c.J1 + c.lay.Joff[li + 1], k.lv[li + 1].g, c.J1 + c.lay.Joff[li], k.lv[li].g, k.C,
                 s);
  }
}

static int check_problem(const lddmm_problem* p) {
  if (!p || !p->template_mask || !p->target_mask || !p->v || !p->workspace) return LDDMM_EINVAL;
  if ((p->template_image == nullptr) != (p->target_image == nullptr)) return LDDMM_EINVAL;
  return LDDMM_OK;
}

static int hip_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LDDMM_OK : LDDMM_EHIP;
}

static int prepare(Ctx& c, const lddmm_problem* p, const lddmm_params* prm, int multilevel) {
  int rc = check_problem(p);
  if (rc) return rc;
  rc = make_config(&p->grid, prm, p->template_image != nullptr, multilevel, &c.cfg);
  if (rc) return rc;
  c.lay = make_layout(c.cfg);
  if (p->workspace_bytes < c.lay.total) return LDDMM_EINVAL;
  bind(c, p->workspace);
  c.alpha = prm->alpha;
  c.gamma = prm->gamma;
  c.sigma = prm->sigma;
  c.guard = prm->guard ? 1 : 0;
  return LDDMM_OK;
}

// ------------------------------------------------- static scratch ----
// The workspace of lddmm_gradient_noalloc: one array per GPU, held from the
// library's load on that GPU until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: only the address that
// hipGetSymbolAddress returns for the current device may reach a kernel.
constexpr size_t kScratchBytes = (size_t)LDDMM_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of the current GPU's scratch array, looked up once per device.
static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LDDMM_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LDDMM_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LDDMM_OK;
}

static int gradient_call(const lddmm_problem* p, const lddmm_params* prm, int32_t kind,
                         float* grad, double* out4, void* stream);

}  // namespace lddmm

using namespace lddmm;

extern "C" {

size_t lddmm_workspace_size(const lddmm_grid* grid, const lddmm_params* params) {
  Config c{};
  if (make_config(grid, params, 1, 1, &c) != LDDMM_OK) {
    // single-level use (energy/gradient) with unchecked descent fields
    if (make_config(grid, params, 1, 0, &c) != LDDMM_OK) return 0;
  }
  Config c1 = c;
  c1.nch = 2;   // size for the largest channel configuration
  return make_layout(c1).total;
}

int lddmm_comp_grid(const lddmm_grid* grid, const lddmm_params* params, int32_t level,
                    int32_t out_P[3]) {
  if (!out_P) return LDDMM_EINVAL;
  int rc = check_params(grid, params, 1);
  if (rc) return rc;
  if (level < 0 || level >= params->n_levels) return LDDMM_EINVAL;
  Level lv[LDDMM_MAX_LEVELS];
  if (!build_levels(grid, params->n_levels, lv)) return LDDMM_EINVAL;
  const Geom& g = lv[params->n_levels - 1 - level].g;
  out_P[0] = g.nx;
  out_P[1] = g.ny;
  out_P[2] = g.nz;
  return LDDMM_OK;
}

int32_t lddmm_trace_rows(const lddmm_params* params) {
  if (!params || params->n_levels < 1 || params->n_levels > LDDMM_MAX_LEVELS) return 0;
  return trace_rows(params);
}

int lddmm_register(lddmm_problem* p, int32_t n_problems, const lddmm_params* prm, void* stream) {
  if (n_problems > 1) return lddmm_register_batched(p, n_problems, prm, nullptr, stream);
  if (n_problems != 1) return LDDMM_EINVAL;
  Ctx c{};
  int rc = prepare(c, p, prm, 1);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  const Config& k = c.cfg;
  const int top = k.L - 1;
  const long long nf = k.lv[top].g.n;
  double* trace = p->trace ? p->trace : c.trace;

  setup_images(c, p, s);
  // initial velocity at the coarsest level: block-average the finest one down
  {
    const float* src = p->v;
    int dst = 1;
    for (int li = top - 1; li >= 0; --li) {
      launch_down2(src, k.lv[li + 1].g, c.v[dst], k.lv[li].g, 3 * k.T, s);
      src = c.v[dst];
      dst ^= 1;
    }
    launch_copy(src, c.v[0], 3 * k.lv[0].g.n * k.T, s);
  }
  launch_level_begin(c.st, prm->step, 0, s);
  for (int li = 0; li <= top; ++li) {
    const Level& L = k.lv[li];
    if (li > 0) {
      // iterate of the previous level -> buffer 0, upsample into buffer 1
      canonicalize(c, 3 * k.lv[li - 1].g.n * k.T, s);
      launch_up2(c.v[0], k.lv[li - 1].g, c.v[1], L.g, 3 * k.T, s);
      launch_copy(c.v[1], c.v[0], 3 * L.g.n * k.T, s);
      launch_level_begin(c.st, prm->step, 1, s);
    }
    level_tables(c, L, s);
    forward_sweep(c, li, c.v[0], c.v[1], false, s);
    decide(c, li, 1, trace, s);
    for (int it = 0; it < prm->iters[li]; ++it) {
      backward_sweep(c, li, c.v[0], c.v[1], nullptr, true, UPD_STEP, nullptr, MODE_GRAD, s, true,
                     g_k_time_batch != 0);
      {
        ProfScope ps(LDDMM_PROF_OTHER, 0, s);
        launch_retry(c.v[0], c.v[1], 3 * L.g.n * k.T, c.st, s);
      }
      forward_sweep(c, li, c.v[0], c.v[1], false, s);
      decide(c, li, 0, trace, s);
    }
  }
  // outputs from the final iterate
  canonicalize(c, 3 * nf * k.T, s);
  launch_copy(c.v[0], p->v, 3 * nf * k.T, s);
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(64), 0, s, c.st, 0, (int)MODE_INIT);
  final_outputs(c, p->phi10, p->phi01, s);
  rc = hip_status();
  if (rc) return rc;
  State hs{};
  if (hipMemcpyAsync(&hs, c.st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess)
    return LDDMM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return LDDMM_EHIP;
  if (hs.nonfinite) {
    const long long N3 = 3LL * k.lv[top].N[0] * k.lv[top].N[1] * k.lv[top].N[2];
    if (p->phi10) launch_fill(p->phi10, N3, NAN, s);
    if (p->phi01) launch_fill(p->phi01, N3, NAN, s);
    if (hipStreamSynchronize(s) != hipSuccess) return LDDMM_EHIP;
    return LDDMM_ENONFINITE;
  }
  if (hs.stopped_any) return LDDMM_WGUARD;
  if (hs.min_det_final <= 0.0) return LDDMM_WFOLD;
  return LDDMM_OK;
}

}  // extern "C"

// ------------------------------------------------------------- batched ----

namespace lddmm {

// Launch arguments of every kernel of one problem at level li, as the single
// problem path builds them (ping-pong map slots, per-step partial buffers).
static void build_pairtab(Ctx& c, int li, PairTab* t) {
  const Config& k = c.cfg;
  const Level& L = k.lv[li];
  const long long n = L.g.n;
  std::memset((void*)t, 0, sizeof(PairTab));
  for (int j = 0; j < k.T; ++j) {
    FwdArgs& a = t->fwd[j];
    a.g = L.g;
    a.vA = c.v[0];
    a.vB = c.v[1];
    a.j = j;
    a.T = k.T;
    a.dt = 1.0f / (float)k.T;
    a.alpha = (float)c.alpha;
    a.gamma = (float)c.gamma;
    a.u_cur = c.u0 + (long long)(j & 1) * 3 * n;
    a.u_next = c.u0 + (long long)((j + 1) & 1) * 3 * n;
    a.J0 = c.J0 + c.lay.Joff[li];
    a.J1 = c.J1 + c.lay.Joff[li];
    a.nch = k.nch;
    a.ch[0] = k.ch[0];
    a.ch[1] = k.nch > 1 ? k.ch[1] : k.ch[0];
    a.w[0] = k.w[0];
    a.w[1] = k.nch > 1 ? k.w[1] : 0.f;
    a.img_ch = k.img_ch;
    a.img_weighted = k.img_weighted;
    a.img_slot = k.img_slot;
    a.J0t_next = c.J0t + (long long)(j + 1 < k.T ? j + 1 : 0) * k.nch * n;
    a.r = c.r;
    a.partR = c.partR + (long long)j * kPartMax;
    a.partD = c.partD;
    a.partI = c.partI;
    a.st = c.st;
    a.zmarch = forward_zmarch(L.g);
    a.staged = forward_staged(L.g);
  }
  for (int j = k.T - 1; j >= -1; --j) {
    BwdArgs& a = t->bwd[j + 1];
    a.g = L.g;
    a.vA = c.v[0];
    a.vB = c.v[1];
    a.vfix = nullptr;
    a.T = k.T;
    a.dt = 1.0f / (float)k.T;
    a.j = j;
    a.u_next = (j == k.T - 1) ? nullptr : c.u1 + (long long)((j + 1) & 1) * 3 * n;
    a.u_cur = j >= 0 ? c.u1 + (long long)(j & 1) * 3 * n : nullptr;
    const int jb = j + 1;
    a.jb = jb <= k.T - 1 ? jb : -1;
    if (a.jb == 0) {
      a.J0t = c.J0 + c.lay.Joff[li] + (long long)k.ch[0] * n;
      a.cstride = k.nch > 1 ? (long long)(k.ch[1] - k.ch[0]) * n : n;
    } else {
      a.J0t = c.J0t + (long long)(a.jb >= 0 ? a.jb : 0) * k.nch * n;
      a.cstride = n;
    }
    a.r = c.r;
    a.nch = k.nch;
    a.w[0] = k.w[0];
    a.w[1] = k.nch > 1 ? k.w[1] : 0.f;
    a.coef = (float)(2.0 / (c.sigma * c.sigma));
    a.b = c.b;
    a.partDet = c.partDet + (long long)(a.jb >= 0 ? a.jb : 0) * kPartMax;
    a.st = c.st;
    a.need_mode = MODE_GRAD;
    a.staged = backward_staged(L.g);
  }
  for (int j = 0; j < k.T; ++j) {
    UpdArgs& u = t->upd[j];
    u.kind = UPD_STEP;
    u.j = j;
    u.vA = c.v[0];
    u.vB = c.v[1];
    u.st = c.st;
    u.need_mode = MODE_GRAD;
  }
  FftLaunch Lf;
  t->fft = make_fft(c, li, MODE_GRAD, &Lf);
  const int nb = forward_tiles(L.g);
  const int nbw = backward_partials(L.g);
  const double h = (double)L.g.h;
  for (int init = 0; init < 2; ++init) {
    DecideArgs& d = t->dec[init];
    d.st = c.st;
    d.partR = c.partR;
    d.partD = c.partD;
    d.partI = c.partI;
    d.partDet = c.partDet;
    d.T = k.T;
    d.nfw = nb;
    d.nbw = nbw;
    d.has_img = k.C > 1;
    d.guard = c.guard;
    d.init = init;
    d.dt = 1.0 / k.T;
    d.h3 = h * h * h;
    d.inv_sigma2 = 1.0 / (c.sigma * c.sigma);
    d.trace = c.trace;
  }
  t->rty.vA = c.v[0];
  t->rty.vB = c.v[1];
  t->rty.count = 3 * n * k.T;
  t->rty.st = c.st;
}

struct BatchPlan {
  BatchRef fwd, bwd, fx, fy, fz, fxi, dec, rty;
  int ex, ey, ez;
  size_t xl, yl, zl;
};

static void batch_offsets(BatchRef& br, int np, const int* tiles, PairTab* const* tabs) {
  br.np = np;
  br.off[0] = 0;
  for (int p = 0; p < np; ++p) {
    br.off[p + 1] = br.off[p] + tiles[p];
    br.tab[p] = tabs[p];
  }
}

}  // namespace lddmm

extern "C" int lddmm_register_batched(lddmm_problem* probs, int32_t n, const lddmm_params* prm,
                                      int32_t* status, void* stream) {
  if (!probs || !prm || n < 1 || n > kMaxBatch) return LDDMM_EINVAL;
  if (prm->flags & LDDMM_FLAG_RK4) return LDDMM_EINVAL;     // batched kernels are first-order
  std::vector<Ctx> cs(n);
  for (int p = 0; p < n; ++p) {
    int rc = prepare(cs[p], &probs[p], prm, 1);
    if (rc) return rc;
  }
  for (int p = 1; p < n; ++p)
    if (cs[p].cfg.nch != cs[0].cfg.nch || cs[p].cfg.L != cs[0].cfg.L) return LDDMM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  const int T = cs[0].cfg.T, L = cs[0].cfg.L, nch = cs[0].cfg.nch;
  std::vector<PairTab> host_tabs((size_t)n * L);
  for (int p = 0; p < n; ++p) {
    Ctx& c = cs[p];
    const Config& k = c.cfg;
    const int top = k.L - 1;
    setup_images(c, &probs[p], s);
    const float* src = probs[p].v;
    int dst = 1;
    for (int li = top - 1; li >= 0; --li) {
      launch_down2(src, k.lv[li + 1].g, c.v[dst], k.lv[li].g, 3 * k.T, s);
      src = c.v[dst];
      dst ^= 1;
    }
    launch_copy(src, c.v[0], 3 * k.lv[0].g.n * k.T, s);
    launch_level_begin(c.st, prm->step, 0, s);
  }
  std::vector<PairTab*> dtabs(n);
  for (int p = 0; p < n; ++p) dtabs[p] = cs[p].ptab;
  for (int li = 0; li < L; ++li) {
    BatchPlan bp{};
    std::vector<int> tf(n), tb(n), tx(n), ty(n), tz(n), tr(n), one(n, 1);
    for (int p = 0; p < n; ++p) {
      Ctx& c = cs[p];
      const Config& k = c.cfg;
      const Level& lv = k.lv[li];
      if (li > 0) {
        canonicalize(c, 3 * k.lv[li - 1].g.n * k.T, s);
        launch_up2(c.v[0], k.lv[li - 1].g, c.v[1], lv.g, 3 * k.T, s);
        launch_copy(c.v[1], c.v[0], 3 * lv.g.n * k.T, s);
        launch_level_begin(c.st, prm->step, 1, s);
      }
      level_tables(c, lv, s);
      PairTab* ht = &host_tabs[(size_t)li * n + p];
      build_pairtab(c, li, ht);
      if (hipMemcpyAsync(c.ptab, ht, sizeof(PairTab), hipMemcpyHostToDevice, s) != hipSuccess)
        return LDDMM_EHIP;
      FftLaunch Lf;
      FftPair tmp = make_fft(c, li, MODE_GRAD, &Lf);
      (void)tmp;
      tf[p] = forward_tiles(lv.g);
      tb[p] = backward_partials(lv.g);
      tx[p] = Lf.x_tiles;
      ty[p] = Lf.y_tiles;
      tz[p] = Lf.z_tiles;
      long long rb = (3 * lv.g.n * k.T + kBlock - 1) / kBlock;   // as launch_retry
      tr[p] = (int)(rb > 4096 ? 4096 : rb);
      bp.ex = std::max(bp.ex, Lf.ex);
      bp.ey = std::max(bp.ey, Lf.ey);
      bp.ez = std::max(bp.ez, Lf.ez);
      bp.xl = std::max(bp.xl, Lf.x_lds);
      bp.yl = std::max(bp.yl, Lf.y_lds);
      bp.zl = std::max(bp.zl, Lf.z_lds);
    }
    batch_offsets(bp.fwd, n, tf.data(), dtabs.data());
    batch_offsets(bp.bwd, n, tb.data(), dtabs.data());
    batch_offsets(bp.fx, n, tx.data(), dtabs.data());
    bp.fxi = bp.fx;
    batch_offsets(bp.fy, n, ty.data(), dtabs.data());
    batch_offsets(bp.fz, n, tz.data(), dtabs.data());
    batch_offsets(bp.dec, n, one.data(), dtabs.data());
    batch_offsets(bp.rty, n, tr.data(), dtabs.data());
    auto forward_all = [&]() {
      for (int j = 0; j < T; ++j) launch_forward_batched(bp.fwd, j, T, nch, s);
    };
    forward_all();
    launch_decide_batched(bp.dec, 1, s);
    for (int it = 0; it < prm->iters[li]; ++it) {
      for (int j = T - 1; j >= -1; --j) {
        launch_backward_batched(bp.bwd, j, T, nch, s);
        const int jb = j + 1;
        if (jb <= T - 1) {
          launch_fft_batched(0, bp.fx, bp.ex, bp.xl, jb, s);
          launch_fft_batched(1, bp.fy, bp.ey, bp.yl, jb, s);
          launch_fft_batched(2, bp.fz, bp.ez, bp.zl, jb, s);
          launch_fft_batched(3, bp.fy, bp.ey, bp.yl, jb, s);
          launch_fft_batched(4, bp.fxi, bp.ex, bp.xl, jb, s);
        }
      }
      launch_retry_batched(bp.rty, s);
      forward_all();
      launch_decide_batched(bp.dec, 0, s);
    }
  }
  // outputs of every problem from its final iterate
  for (int p = 0; p < n; ++p) {
    Ctx& c = cs[p];
    const Config& k = c.cfg;
    const int top = k.L - 1;
    const long long nf = k.lv[top].g.n;
    lddmm_problem* pr = &probs[p];
    canonicalize(c, 3 * nf * k.T, s);
    launch_copy(c.v[0], pr->v, 3 * nf * k.T, s);
    hipLaunchKernelGGL(k_set_base, dim3(1), dim3(64), 0, s, c.st, 0, (int)MODE_INIT);
    final_outputs(c, pr->phi10, pr->phi01, s);
    if (pr->trace) {
      const int rows = trace_rows(prm);
      hipMemcpyAsync(pr->trace, c.trace, sizeof(double) * 8 * rows, hipMemcpyDeviceToDevice, s);
    }
  }
  int rc = hip_status();
  if (rc) return rc;
  std::vector<State> hs(n);
  for (int p = 0; p < n; ++p)
    if (hipMemcpyAsync(&hs[p], cs[p].st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess)
      return LDDMM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return LDDMM_EHIP;
  int worst = LDDMM_OK;
  for (int p = 0; p < n; ++p) {
    const Config& k = cs[p].cfg;
    int st = LDDMM_OK;
    if (hs[p].nonfinite) {
      const long long N3 = 3LL * k.lv[k.L - 1].N[0] * k.lv[k.L - 1].N[1] * k.lv[k.L - 1].N[2];
      if (probs[p].phi10) launch_fill(probs[p].phi10, N3, NAN, s);
      if (probs[p].phi01) launch_fill(probs[p].phi01, N3, NAN, s);
      st = LDDMM_ENONFINITE;
    } else if (hs[p].stopped_any) {
      st = LDDMM_WGUARD;
    } else if (hs[p].min_det_final <= 0.0) {
      st = LDDMM_WFOLD;
    }
    if (status) status[p] = st;
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (worst >= 0 && st > worst) worst = st;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return LDDMM_EHIP;
  return worst;
}

extern "C" {

int lddmm_energy(const lddmm_problem* p, const lddmm_params* prm, double* out4, void* stream) {
  if (!out4) return LDDMM_EINVAL;
  Ctx c{};
  int rc = prepare(c, p, prm, 0);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  setup_images(c, p, s);
  launch_level_begin(c.st, 1.0, 0, s);
  level_tables(c, c.cfg.lv[0], s);
  forward_sweep(c, 0, p->v, p->v, false, s);
  decide(c, 0, 1, c.trace, s);
  launch_energy_out(c.st, out4, s);
  return hip_status();
}

int lddmm_gradient(const lddmm_problem* p, const lddmm_params* prm, int32_t kind, float* grad,
                   double* out4, void* stream) {
  return gradient_call(p, prm, kind, grad, out4, stream);
}

int lddmm_gradient_noalloc(const lddmm_problem* p, const lddmm_params* prm, int32_t kind,
                           float* grad, double* out4, void* stream) {
  if (!p || !prm) return LDDMM_EINVAL;
  Config cfg{};
  int rc = make_config(&p->grid, prm, p->template_image != nullptr, 0, &cfg);
  if (rc) return rc;
  if (make_layout(cfg).total > kScratchBytes) return LDDMM_ESCRATCH;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  lddmm_problem q = *p;
  q.workspace = ws;
  q.workspace_bytes = kScratchBytes;
  return gradient_call(&q, prm, kind, grad, out4, stream);
}

}  // extern "C"

namespace lddmm {

static int gradient_call(const lddmm_problem* p, const lddmm_params* prm, int32_t kind,
                         float* grad, double* out4, void* stream) {
  if (!grad || !out4) return LDDMM_EINVAL;
  if (kind != LDDMM_GRAD_V && kind != LDDMM_GRAD_L2) return LDDMM_EINVAL;
  if (kind == LDDMM_GRAD_L2 && prm && (prm->flags & LDDMM_FLAG_RK4)) return LDDMM_EINVAL;
  Ctx c{};
  int rc = prepare(c, p, prm, 0);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  setup_images(c, p, s);
  launch_level_begin(c.st, 1.0, 0, s);
  if (kind == LDDMM_GRAD_L2) {
    launch_fill((float*)c.misc, 2, 0.f, s);   // radius, overflow flag (zero bits)
    exact_gradient(c, p->v, grad, s);
    launch_energy_out_checked(c.st, c.misc + 1, out4, s);
    return hip_status();
  }
  level_tables(c, c.cfg.lv[0], s);
  forward_sweep(c, 0, p->v, p->v, false, s);
  decide(c, 0, 1, c.trace, s);
  launch_energy_out(c.st, out4, s);
  backward_sweep(c, 0, p->v, p->v, p->v, true, UPD_WRITE_G, grad, -1, s);
  return hip_status();
}

}  // namespace lddmm

extern "C" {

int lddmm_apply(const lddmm_grid* grid, const float* u, const void* src, int32_t interp,
                int32_t dtype, void* dst, void* stream) {
  if (!grid || !u || !src || !dst) return LDDMM_EINVAL;
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return LDDMM_EINVAL;
  if (!(grid->spacing > 0.0)) return LDDMM_EINVAL;
  if (interp != LDDMM_INTERP_LINEAR && interp != LDDMM_INTERP_NEAREST) return LDDMM_EINVAL;
  if (dtype != LDDMM_F32 && dtype != LDDMM_I32) return LDDMM_EINVAL;
  if (interp == LDDMM_INTERP_LINEAR && dtype != LDDMM_F32) return LDDMM_EINVAL;
  hipGetLastError();
  launch_apply(u, grid->nx, grid->ny, grid->nz, (float)(1.0 / grid->spacing), src, interp, dtype,
               dst, (hipStream_t)stream);
  return hip_status();
}

size_t lddmm_smooth_workspace_size(const int32_t P[3]) {
  if (!P) return 0;
  for (int d = 0; d < 3; ++d)
    if (P[d] < 2 || P[d] > LDDMM_MAX_DIM || !is_7smooth(P[d])) return 0;
  const size_t nspec = (size_t)((P[0] / 2 + 1 + 15) / 16 * 16) * P[1] * P[2];
  size_t off = align_up(sizeof(State));
  for (int d = 0; d < 3; ++d) off = align_up(off + sizeof(float2) * P[d]);
  for (int d = 0; d < 3; ++d) off = align_up(off + sizeof(double) * P[d]);
  off = align_up(off + sizeof(float) * 3 * (size_t)P[0] * P[1] * P[2]);
  off = align_up(off + sizeof(float2) * 3 * nspec);
  return off;
}

int lddmm_smooth(const int32_t P[3], double spacing, double alpha, double gamma, const float* b,
                 float* out, void* workspace, size_t workspace_bytes, void* stream) {
  const size_t need = lddmm_smooth_workspace_size(P);
  if (need == 0 || !b || !out || !workspace || workspace_bytes < need) return LDDMM_EINVAL;
  if (!(spacing > 0.0) || !(alpha >= 0.0) || !(gamma > 0.0)) return LDDMM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  Ctx c{};
  Level L{};
  L.g = make_geom(P[0], P[1], P[2], spacing);
  if (!make_plan(P[0], &L.px) || !make_plan(P[1], &L.py) || !make_plan(P[2], &L.pz))
    return LDDMM_EINVAL;
  c.cfg.lv[0] = L;
  c.cfg.L = 1;
  char* w = (char*)workspace;
  size_t off = 0;
  c.st = (State*)(w + off);
  off = align_up(sizeof(State));
  for (int d = 0; d < 3; ++d) {
    c.tw[d] = (float2*)(w + off);
    off = align_up(off + sizeof(float2) * P[d]);
  }
  for (int d = 0; d < 3; ++d) {
    c.lam[d] = (double*)(w + off);
    off = align_up(off + sizeof(double) * P[d]);
  }
  c.b = (float*)(w + off);
  off = align_up(off + sizeof(float) * 3 * (size_t)L.g.n);
  c.S = (float2*)(w + off);
  c.alpha = alpha;
  c.gamma = gamma;
  launch_level_begin(c.st, 1.0, 0, s);
  level_tables(c, L, s);
  launch_copy(b, c.b, 3 * L.g.n, s);
  UpdArgs u{};
  u.kind = UPD_WRITE_KB;
  u.out = out;
  u.st = c.st;
  u.need_mode = -1;
  smooth_and_update(c, 0, u, -1, s);
  return hip_status();
}

int lddmm_make_mask(const lddmm_grid* grid, const float* image, float tau, float* mask,
                    float* masked_image, void* stream) {
  if (!grid || !image || !mask) return LDDMM_EINVAL;
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return LDDMM_EINVAL;
  hipGetLastError();
  launch_make_mask(image, (long long)grid->nx * grid->ny * grid->nz, tau, mask, masked_image,
                   (hipStream_t)stream);
  return hip_status();
}

int lddmm_copy(const float* src, float* dst, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!src || !dst))) return LDDMM_EINVAL;
  if (n == 0) return LDDMM_OK;
  (void)hipGetLastError();
  launch_copy(src, dst, (long long)n, (hipStream_t)stream);
  return hip_status();
}

int lddmm_set_tunable(int32_t which, int32_t value) {
  if (which == LDDMM_TUNE_SWEEP_BLOCKS) {
    if (value < 1) return LDDMM_EINVAL;
    set_sweep_blocks(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_FWD_TILES) {
    if (value < 0) return LDDMM_EINVAL;
    set_fwd_tiles(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_STAGED_MIN_BLOCKS) {
    if (value < 1) return LDDMM_EINVAL;
    set_staged_min_blocks(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_FWD_STAGED_MIN_BLOCKS) {
    if (value < 1) return LDDMM_EINVAL;
    set_fwd_staged_min_blocks(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_FFT_FUSED_LDS) {
    if (value < 0) return LDDMM_EINVAL;
    set_fft_fused_lds(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_K_TIME_BATCH) {
    if (value < 0 || value > 1) return LDDMM_EINVAL;
    set_k_time_batch(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_FFT_X_ELEMS) {
    if (value < 1) return LDDMM_EINVAL;
    set_fft_x_elems(value);
    return LDDMM_OK;
  }
  if (which == LDDMM_TUNE_FFT_COLS || which == LDDMM_TUNE_FFT_ZCOLS) {
    if (value < 1) return LDDMM_EINVAL;
    set_fft_cols(which == LDDMM_TUNE_FFT_COLS ? 0 : 1, value);
    return LDDMM_OK;
  }
  return LDDMM_EINVAL;
}

int lddmm_profile_begin(uint32_t class_mask, int64_t min_voxels) {
  g_prof_min_vox = min_voxels;
  g_prof_rec.clear();
  g_prof_used = 0;
  g_prof_mask = class_mask & ((1u << LDDMM_PROF_CLASSES) - 1);
  return LDDMM_OK;
}

int lddmm_profile_end(double* ms_total, int64_t* launches, int64_t* voxels) {
  double ms[LDDMM_PROF_CLASSES] = {0};
  int64_t cnt[LDDMM_PROF_CLASSES] = {0}, vox[LDDMM_PROF_CLASSES] = {0};
  int rc = LDDMM_OK;
  for (const ProfRec& r : g_prof_rec) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      rc = LDDMM_EHIP;
      continue;
    }
    ms[r.cls] += t;
    cnt[r.cls] += 1;
    vox[r.cls] += r.vox;
  }
  for (int k = 0; k < LDDMM_PROF_CLASSES; ++k) {
    if (ms_total) ms_total[k] = ms[k];
    if (launches) launches[k] = cnt[k];
    if (voxels) voxels[k] = vox[k];
  }
  g_prof_mask = 0;
  g_prof_rec.clear();
  g_prof_used = 0;
  return rc;
}

const char* lddmm_strerror(int code) {
  switch (code) {
    case LDDMM_OK: return "ok";
    case LDDMM_EINVAL: return "invalid argument";
    case LDDMM_EHIP: return "HIP runtime or launch error";
    case LDDMM_ENONFINITE: return "energy is not finite";
    case LDDMM_WFOLD: return "warning: Jacobian determinant <= 0 (fold) seen";
    case LDDMM_WGUARD: return "warning: step guard stopped a level after repeated halvings";
    case LDDMM_ESCRATCH:
      return "problem needs more workspace than the static scratch of lddmm_gradient_noalloc";
    default: return "unknown status";
  }
}

}  // extern "C"

// ------------------------------------------------- warm-start expansion ----

namespace lddmm {

// planar[ch][vox] = scale * out[vox][ch]
__global__ void k_unpack_channels(const float* out, long long nvox, int C, float scale,
                                  float* planar) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * C) return;
  const long long ch = i / nvox;
  const long long p = i - ch * nvox;
  planar[i] = scale * out[p * C + ch];
}

}  // namespace lddmm

extern "C" int lddmm_cnn_expand_velocity(const float* out, int32_t T, int32_t d, int32_t h,
                                         int32_t w, float scale, float* v, float* scratch,
                                         void* stream) {
  if (!out || !v || !scratch || T < 1 || T > LDDMM_MAX_T || d < 2 || h < 2 || w < 2 ||
      4 * std::max(d, std::max(h, w)) > LDDMM_MAX_DIM)
    return LDDMM_EINVAL;
  const long long nc = (long long)d * h * w;
  if (3LL * T * 64 * nc >= (1LL << 31)) return LDDMM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const Geom g0 = make_geom(w, h, d, 1.0), g1 = make_geom(2 * w, 2 * h, 2 * d, 1.0),
             g2 = make_geom(4 * w, 4 * h, 4 * d, 1.0);
  float* mid = scratch;                          // 3T fields on the 2x grid
  float* planar = scratch + 3LL * T * g1.n;      // 3T fields on the coarse grid
  hipGetLastError();
  const long long total = nc * 3 * T;
  hipLaunchKernelGGL(k_unpack_channels, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     out, nc, 3 * T, scale, planar);
  launch_up2(planar, g0, mid, g1, 3 * T, s);
  launch_up2(mid, g1, v, g2, 3 * T, s);
  return hip_status();
}

// swe_nh_api.cpp -- host side of the C ABI declared in include/swe_nh.h:
// configuration checks, workspace layout, channel/tile tables, kernel
// sequencing and hipGraph capture of the time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "swe_nh.h"
#include "swe_nh_2d.h"
#include "swe_nh_cnn.h"
#include "swe_nh_kernels.h"

using namespace swenh;

namespace {

// bump allocator over the caller's workspace (base == nullptr: size only)
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

}  // namespace

constexpr int GSTEPS = 8;  // steps per graph launch on the fused 1D path (even)
constexpr int TIME_BATCH = 50;  // stage launches per graph in swe_nh_time_stage

struct swe_nh_ctx {
  swe_nh_config cfg{};
  std::vector<int64_t> offsets;
  std::vector<swe_nh_body> bodies;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  int nch = 0;
  int64_t ncells = 0;
  std::string err;
  // device scalars
  int* status = nullptr;
  int* step = nullptr;
  int* n_act = nullptr;
  int* conv = nullptr;
  int* iters = nullptr;
  double* norms = nullptr;
  double* rel = nullptr;
  double* part = nullptr;
  double* part_b = nullptr;
  int nparts = 0;
  double* stage_t = nullptr;
  double* stage_dt = nullptr;
  // 1D
  K1D k1{};
  std::vector<int4> tiles;
  double *ht = nullptr, *mt = nullptr, *kt = nullptr;
  uint8_t* mask_ws = nullptr;
  TriLevels<double> T64{};
  TriLevels<float> T32{};
  TriLevels<double> T1{};  // level-1 system of the tile-fused step
  int* n1 = nullptr;       // its row count (2 per tile)
  // 2D
  Ctx2D c2{};
  // graph of one step (fused 1D path: two, alternating the state buffers)
  hipGraphExec_t gexec = nullptr;
  hipGraphExec_t gexec2 = nullptr;
  hipGraphExec_t gexecN = nullptr;  // fused 1D path: GSTEPS steps in one graph
  // adaptive 2D (5-point): the step without the multigrid's launches, chosen
  // from the active-tile count of an earlier call (read back through pinned
  // memory once an event says the copy is done; never waited for)
  hipGraphExec_t gexecT = nullptr;
  int* tiles_host = nullptr;
  hipEvent_t tiles_ev = nullptr;
  bool tiles_pending = false;
  bool mg_graph = false;
  const void* gkey[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t steps_taken = 0;
};

namespace {

int fail(swe_nh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, SWE_NH_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

int check_config(const swe_nh_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return SWE_NH_EINVAL;
  };
  if (!c) return bad("null config");
  if (c->dim != 1 && c->dim != 2) return bad("dim must be 1 or 2");
  if (!(c->dx > 0.0) || (c->dim == 2 && !(c->dy > 0.0))) return bad("dx, dy must be > 0");
  if (!(c->g > 0.0) || !(c->rho > 0.0)) return bad("g and rho must be > 0");
  if (!(c->cfl > 0.0) && !(c->dt_fixed > 0.0)) return bad("need cfl > 0 or dt_fixed > 0");
  if (c->crit < 0 || c->crit > SWE_NH_CRIT_NONE) return bad("unknown criterion");
  if (c->enlarge < 0 || c->enlarge > 64) return bad("enlarge must be in [0, 64]");
  if (c->tile1d != 0 && (c->tile1d < 32 || c->tile1d > TILE_MAX))
    return bad("tile1d must be 0 or in [32, 512]");
  if (c->step1d_form != 0 && c->step1d_form != 1) return bad("step1d_form must be 0 or 1");
  if (c->tensor2d != 0 && c->tensor2d != 1) return bad("tensor2d must be 0 or 1");
  if (c->tensor2d && c->dim != 2) return bad("tensor2d is a 2D operator");
  if (c->precision != 0 && c->precision != 1) return bad("precision must be 0 or 1");
  if (!c->depth_static) return bad("depth_static is required");
  if (!c->bodies) return bad("bodies is required");
  if (c->dim == 1) {
    if (c->batch < 1) return bad("batch must be >= 1");
    if (c->batch > 1 && !c->offsets) return bad("offsets required when batch > 1");
    if (c->batch == 1 && !c->offsets && c->nx < 4) return bad("a channel needs >= 4 cells");
    if (c->offsets) {
      if (c->offsets[0] != 0) return bad("offsets[0] must be 0");
      for (int b = 0; b < c->batch; b++)
        if (c->offsets[b + 1] - c->offsets[b] < 4) return bad("a channel needs >= 4 cells");
      if (c->offsets[c->batch] >= (int64_t(1) << 31)) return bad("too many cells");
    }
    if (c->precision == 1 && c->max_iter < 1) return bad("max_iter >= 1 for refinement");
  } else {
    if (c->nx < 4 || c->ny < 4) return bad("2D grid needs nx, ny >= 4");
    if ((int64_t)c->nx * c->ny >= (int64_t(1) << 31)) return bad("grid too large");
    if (c->max_iter < 1) return bad("max_iter must be >= 1");
    if (!(c->tol > 0.0)) return bad("tol must be > 0");
    if (c->tensor2d) {
      int lnx[MG_MAXL + 1], lny[MG_MAXL + 1];
      if (mg_plan_levels(c->nx, c->ny, lnx, lny) == 0)
        return bad("tensor2d needs a grid that coarsens by 2 x 2 aggregation to <= 4096 cells");
    }
  }
  return SWE_NH_OK;
}

int64_t total_cells(const swe_nh_config* c) {
  if (c->dim == 2) return (int64_t)c->nx * c->ny;
  return c->offsets ? c->offsets[c->batch] : c->nx;
}

int n_channels(const swe_nh_config* c) { return c->dim == 2 ? 1 : c->batch; }

bool fused_step(const swe_nh_config* c) {
  return c->dim == 1 && c->enlarge <= fused_max_enlarge();
}

// cells per 1D tile: the configured number, else a window capacity of 128
// cells, or of 512 when tiles of 128 would give more than 1024 tiles.  The
// fused step's window adds 6 + e cells on each side, so there the tile is the
// capacity less twice that: the window then fills whole wavefronts.
int tile_of(const swe_nh_config* c) {
  if (c->tile1d > 0) return c->tile1d;
  const int64_t N = c->dim == 2 ? (int64_t)c->nx * c->ny : (c->offsets ? c->offsets[c->batch] : c->nx);
  const int cap = N <= 256 * 512 ? 128 : 512;
  return fused_step(c) ? cap - 2 * (6 + c->enlarge) : cap;
}

// LDS capacity of the tile kernels that hold a tile of tile_of(c) cells
int cap_of(const swe_nh_config* c) {
  const int t = tile_of(c);
  return t <= 128 ? 128 : t <= 256 ? 256 : 512;
}

// wave-speed slots per channel: a power of two, about one slot per 32 tiles
// of the longest channel (1 in 2D, where the tiles publish their own maxima)
int speed_slots(const swe_nh_config* c) {
  if (c->dim != 1) return 1;
  int64_t nmax = 0;
  for (int b = 0; b < n_channels(c); b++)
    nmax = std::max<int64_t>(nmax, c->offsets ? c->offsets[b + 1] - c->offsets[b] : c->nx);
  const int64_t tiles = (nmax + tile_of(c) - 1) / tile_of(c);
  int s = 1;
  while (s < SPEED_SLOTS_MAX && (int64_t)s * 32 < tiles) s *= 2;
  return s;
}

// per tile: (channel, first cell, packed offset of the channel, cells of the
// channel), so that a block has every index it needs from one load
void tile_table(const swe_nh_config* c, std::vector<int4>* tiles, std::vector<int>* first) {
  const int nch = n_channels(c);
  const int T = tile_of(c);
  for (int b = 0; b < nch; b++) {
    const int64_t n = c->offsets ? c->offsets[b + 1] - c->offsets[b] : c->nx;
    first->push_back((int)tiles->size());
    const int off = c->offsets ? (int)c->offsets[b] : 0;
    for (int64_t s = 0; s < n; s += T) tiles->push_back(make_int4(b, (int)s, off, (int)n));
  }
}

template <typename R>
void plan_levels(TriLevels<R>* T, int64_t N, Carve& cv, int* nbuf) {
  int64_t nm = N;
  int l = 0;
  for (;;) {
    T->nmax[l] = nm;
    T->dg[l] = cv.take<R>(nm);
    T->up[l] = cv.take<R>(nm);
    T->rh[l] = cv.take<R>(nm);
    T->x[l] = cv.take<R>(nm);
    l++;
    if (nm <= TRI_ROWS || l == TRI_MAX_LEVELS) break;
    nm = 2 * ((nm + TRI_ROWS - 1) / TRI_ROWS);
  }
  T->nlev = l;
  T->n = nbuf;
}

// lays out the workspace; returns its size (ctx == nullptr / base == nullptr: size only)
size_t plan(const swe_nh_config* c, char* base, swe_nh_ctx* ctx) {
  Carve cv{base};
  const int nch = n_channels(c);
  const int64_t N = total_cells(c);
  std::vector<int4> tiles;
  std::vector<int> first;
  tile_table(c, &tiles, &first);
  const int ntiles = (int)tiles.size();
  swe_nh_ctx tmp;
  swe_nh_ctx* x = ctx ? ctx : &tmp;
  K1D& P = x->k1;
  P.ch = cv.take<Chan>(nch);
  P.tiles = cv.take<int4>(ntiles);
  P.first_tile = cv.take<int>(nch);
  P.t = cv.take<double>(2 * (size_t)nch);
  P.dt = cv.take<double>(nch);
  P.smax = cv.take<unsigned long long>(speed_at(2 * nch, 0, speed_slots(c)));
  x->stage_t = cv.take<double>(nch);
  x->stage_dt = cv.take<double>(nch);
  x->status = cv.take<int>(1);
  x->step = cv.take<int>(2);
  x->n_act = cv.take<int>(1);
  x->conv = cv.take<int>(1);
  x->iters = cv.take<int>(1);
  x->norms = cv.take<double>(2);
  x->rel = cv.take<double>(1);
  int* nbuf64 = cv.take<int>(TRI_MAX_LEVELS);
  int* nbuf32 = cv.take<int>(TRI_MAX_LEVELS);
  int* nbuf1 = cv.take<int>(TRI_MAX_LEVELS);
  P.n_acc = cv.take<int>(2);
  x->n1 = cv.take<int>(1);
  if (c->dim == 1) {
    P.tile_cnt = cv.take<int>(ntiles);
    P.tile_off = cv.take<int>(ntiles);
    P.act_cell = cv.take<int>(N);
    P.act_chan = cv.take<int>(N);
    x->ht = cv.take<double>(N);
    x->mt = cv.take<double>(N);
    x->kt = cv.take<double>(N);
    x->mask_ws = cv.take<uint8_t>(N);
    plan_levels(&x->T64, N, cv, nbuf64);
    if (c->precision == 1) plan_levels(&x->T32, N, cv, nbuf32);
    if (fused_step(c)) {
      plan_levels(&x->T1, 2 * (int64_t)ntiles, cv, nbuf1);
      P.zw = cv.take<double>((size_t)ZW_N * ntiles * cap_of(c));
      P.dg1 = x->T1.dg[0];
      P.up1 = x->T1.up[0];
      P.rh1 = x->T1.rh[0];
      P.x1 = x->T1.x[0];
      // tagged words of the one-kernel step: counts, rows, solution
      P.tw = cv.take<unsigned long long>(17 * (size_t)ntiles);
      P.tag1 = cv.take<unsigned>(1);
      P.ctab = cv.take<double>(CTAB_N * (size_t)nch);
      P.mlist = cv.take<int>(ntiles);
      P.mcount = cv.take<int>(1);
      P.l1s = cv.take<double>(4 * (size_t)ntiles);
      P.sweeps = cv.take<int>(2);
      P.berr = cv.take<unsigned long long>(2);
    }
    x->nparts = resid_blocks(N);
    x->part = cv.take<double>(x->nparts);
    x->part_b = cv.take<double>(x->nparts);
  } else {
    plan2d(c, cv.base, &cv.off, &x->c2);
  }
  P.status = x->status;
  P.step = x->step;
  P.n_act = x->n_act;
  return cv.off + 256;
}

int decide_mask_mode(const swe_nh_config* c, int first_step) {
  const bool w = (c->crit == SWE_NH_CRIT_W || c->crit == SWE_NH_CRIT_W_X);
  if (c->crit == SWE_NH_CRIT_GLOBAL || (w && first_step && c->first_global)) return 1;
  if (c->crit == SWE_NH_CRIT_NONE) return 2;
  return 0;
}

// ------------------------------------------------------------------ 1D ---

void solve1d(swe_nh_ctx* c, hipStream_t s, int with_residual) {
  const int64_t N = c->ncells;
  if (c->cfg.precision == 0) {
    launch_tri_solve(c->T64, c->n_act, nullptr, s);
    if (with_residual) {
      launch_resid1d(c->T64.dg[0], c->T64.up[0], c->T64.rh[0], c->T64.x[0], c->n_act, N, nullptr,
                     c->part, 1, c->part_b, nullptr, s);
      launch_resid_final(c->part, c->part_b, c->nparts, 1, c->cfg.tol, c->norms, c->rel,
                         c->iters, nullptr, 1, s);
    }
    return;
  }
  // FP32 solves of A e = r with FP64 residuals, x += e, until ||r|| <= tol ||b||
  TriLevels<float>& T = c->T32;
  launch_cast_sys(c->T64.dg[0], c->T64.up[0], c->T64.rh[0], c->n_act, N, T.dg[0], T.up[0],
                  T.rh[0], s);
  launch_resid1d(c->T64.dg[0], c->T64.up[0], c->T64.rh[0], nullptr, c->n_act, N, nullptr, c->part,
                 1, c->part_b, nullptr, s);
  launch_resid_final(c->part, c->part_b, c->nparts, 0, c->cfg.tol, c->norms, c->rel, c->iters,
                     c->conv, 1, s);
  launch_fill_i32(c->conv, 1, 0, s);
  for (int j = 1; j <= c->cfg.max_iter; j++) {
    launch_tri_solve(T, c->n_act, c->conv, s);
    launch_refine_update(T.x[0], c->T64.x[0], c->n_act, N, j == 1, c->conv, s);
    launch_resid1d(c->T64.dg[0], c->T64.up[0], c->T64.rh[0], c->T64.x[0], c->n_act, N, T.rh[0],
                   c->part, 0, nullptr, c->conv, s);
    launch_resid_final(c->part, nullptr, c->nparts, j, c->cfg.tol, c->norms, c->rel, c->iters,
                       c->conv, 0, s);
  }
  launch_flag_noconv(c->conv, c->status, s);
}

// fused FP64 step from (h, hu, hw) into (hn, hun, hwn)
void enqueue_fused1d(swe_nh_ctx* c, hipStream_t s, const double* h, const double* hu,
                     const double* hw, double* hn, double* hun, double* hwn, double* p,
                     uint8_t* mask, int par) {
  K1D& P = c->k1;
  uint8_t* M = mask ? mask : c->mask_ws;
  launch_step1d(P, h, hu, hw, hn, hun, hwn, M, p, par, s);
  if (P.onepass) return;  // the step kernel also solved and projected
  if (!level1_local(P)) {
    if (level1_per_channel(P))
      launch_level1_chan(P, s);
    else
      launch_tri_solve(c->T1, c->n1, nullptr, s);
  }
  launch_apply1d(P, M, hun, hwn, p, par, s);
}

void enqueue_step1d(swe_nh_ctx* c, hipStream_t s, double* h, double* hu, double* hw, double* p,
                    uint8_t* mask) {
  K1D& P = c->k1;
  uint8_t* M = mask ? mask : c->mask_ws;
  const int64_t N = c->ncells;

  launch_speed1d(P, h, hu, hw, s);
  launch_pred1d(P, h, hu, hw, c->ht, c->mt, c->kt, P.t, P.dt, 1, s);
  launch_mask1d(P, c->ht, c->mt, c->kt, P.t, P.dt, -1, M, h, hu, hw, p, 1, s);
  launch_scan(P.tile_cnt, P.tile_off, P.ntiles, c->n_act, s);
  if (c->cfg.crit != SWE_NH_CRIT_NONE) {
    launch_compact1d(P, M, s);
    launch_assemble1d(P, N, c->ht, c->mt, c->kt, M, P.t, P.dt, c->T64.dg[0], c->T64.up[0],
                      c->T64.rh[0], s);
    solve1d(c, s, 0);
    launch_correct1d(P, N, c->ht, c->mt, c->kt, M, P.t, P.dt, c->T64.x[0], hu, hw, p, s);
  }
  launch_advance(P, c->nch, s);
}

int upload_stage_times(swe_nh_ctx* c, const double* t_host, const double* dt_host) {
  std::vector<double> z(c->nch, 0.0);
  HIPCHK(c, hipMemcpyAsync(c->stage_t, t_host, sizeof(double) * c->nch, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->stage_dt, dt_host ? dt_host : z.data(), sizeof(double) * c->nch,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the host arrays are transient
  return SWE_NH_OK;
}

int reset_status(swe_nh_ctx* c) {
  launch_fill_i32(c->status, 1, 0, c->stream);
  return SWE_NH_OK;
}

int status_code(int bits) {
  if (bits & ST_NAN) return SWE_NH_ENAN;
  if (bits & ST_DRY) return SWE_NH_EDRY;
  if (bits & ST_ABORT) return SWE_NH_EHIP;  // a device-side wait timed out
  if (bits & ST_NOCONV) return SWE_NH_ENOCONV;
  return SWE_NH_OK;
}

int after_launch(swe_nh_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, SWE_NH_EHIP, std::string("launch: ") + hipGetErrorString(e));
  return SWE_NH_OK;
}

// adaptive 2D steps with the 5-point operator choose per call between a step
// graph with the multigrid's launches and one without (the tile solver then
// takes every step, as it can at any active-tile count)
bool mg_choice(const swe_nh_ctx* c) {
  return c->cfg.dim == 2 && c->c2.mg_levels > 0 && !c->c2.tensor &&
         c->cfg.crit != SWE_NH_CRIT_GLOBAL && c->cfg.crit != SWE_NH_CRIT_NONE;
}

// captures the work enqueued by f on the private stream into an executable graph
template <typename F>
int capture_graph(swe_nh_ctx* c, F f, hipGraphExec_t* out) {
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
  f(c->cap);
  hipGraph_t g = nullptr;
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, SWE_NH_EHIP,
                std::string("capture: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, SWE_NH_EHIP, std::string("instantiate: ") + hipGetErrorString(e3));
  return SWE_NH_OK;
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

size_t swe_nh_workspace_bytes(const swe_nh_config* cfg) {
  if (check_config(cfg, nullptr) != SWE_NH_OK) return 0;
  return plan(cfg, nullptr, nullptr);
}

int swe_nh_init(const swe_nh_config* cfg, void* workspace, size_t bytes, void* stream,
                swe_nh_ctx** out) {
  if (!out) return SWE_NH_EINVAL;
  *out = nullptr;
  std::string why;
  if (check_config(cfg, &why) != SWE_NH_OK) {
    fprintf(stderr, "swe_nh_init: %s\n", why.c_str());
    return SWE_NH_EINVAL;
  }
  const size_t need = plan(cfg, nullptr, nullptr);
  if (!workspace || bytes < need) return SWE_NH_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return SWE_NH_EINVAL;
  swe_nh_ctx* c = new swe_nh_ctx();
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  c->nch = n_channels(cfg);
  c->ncells = total_cells(cfg);
  if (cfg->offsets) c->offsets.assign(cfg->offsets, cfg->offsets + cfg->batch + 1);
  c->bodies.assign(cfg->bodies, cfg->bodies + c->nch);
  c->cfg.offsets = c->offsets.empty() ? nullptr : c->offsets.data();
  c->cfg.bodies = c->bodies.data();
  plan(&c->cfg, static_cast<char*>(workspace), c);
  hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return SWE_NH_EHIP;
  }
  if (mg_choice(c)) {
    e = hipHostMalloc((void**)&c->tiles_host, sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->tiles_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      swe_nh_destroy(c);
      return SWE_NH_EHIP;
    }
  }
  // channel table
  std::vector<Chan> ch(c->nch);
  for (int b = 0; b < c->nch; b++) {
    Chan& q = ch[b];
    const swe_nh_body& bd = c->bodies[b];
    q.off = cfg->dim == 2 ? 0 : (cfg->offsets ? cfg->offsets[b] : 0);
    q.n = cfg->dim == 2 ? cfg->nx : (int)(cfg->offsets ? cfg->offsets[b + 1] - cfg->offsets[b] : cfg->nx);
    q.kind = bd.kind;
    q.law = bd.law;
    q.pad = 0;
    q.amp = bd.amp;
    q.len = bd.len;
    q.x0 = bd.x0;
    q.y0 = bd.y0;
    q.dir = bd.dir;
    for (int j = 0; j < 5; j++) q.q[j] = bd.q[j];
  }
  std::vector<int> first;
  tile_table(&c->cfg, &c->tiles, &first);
  K1D& P = c->k1;
  P.ds = cfg->depth_static;
  P.dx = cfg->dx;
  P.g = cfg->g;
  P.rho = cfg->rho;
  P.cfl = cfg->cfl;
  P.dt_fixed = cfg->dt_fixed;
  P.k_nh = cfg->k_nh;
  P.crit = cfg->crit;
  P.enlarge = cfg->enlarge;
  P.first_global = cfg->first_global;
  P.ntiles = (int)c->tiles.size();
  P.tile = tile_of(cfg);
  P.cap = cap_of(cfg);
  P.nch = c->nch;
  P.max_ch_tiles = 0;
  for (int b = 0; b < (int)first.size(); b++) {
    const int end = b + 1 < (int)first.size() ? first[b + 1] : P.ntiles;
    P.max_ch_tiles = std::max(P.max_ch_tiles, end - first[b]);
  }
  P.nslot = speed_slots(cfg);
  P.fused = fused_step(cfg) ? 1 : 0;
  P.onepass = 0;
  P.keep_speed = 0;
  P.refine = (P.fused && cfg->precision == 1) ? 1 : 0;
  P.max_sweeps = cfg->max_iter;
  P.tol = cfg->tol;
  P.iters_out = c->iters;
  P.rel_out = c->rel;
  const int n1 = 2 * P.ntiles;
  std::vector<double> zeros(c->nch, 0.0);
  std::vector<unsigned long long> zu(speed_at(2 * c->nch, 0, P.nslot), 0ull);
  int zi[TRI_MAX_LEVELS * 2] = {0};
  int rc = SWE_NH_OK;
#define INIT_COPY(dst, src, bytes)                                                  \
  if (rc == SWE_NH_OK && hipMemcpy((void*)(dst), (src), (bytes), hipMemcpyHostToDevice) != \
                             hipSuccess)                                           \
    rc = SWE_NH_EHIP;
  INIT_COPY(P.ch, ch.data(), sizeof(Chan) * c->nch);
  if (cfg->dim == 1) {
    INIT_COPY(P.tiles, c->tiles.data(), sizeof(int4) * c->tiles.size());
    INIT_COPY(P.first_tile, first.data(), sizeof(int) * first.size());
  }
  INIT_COPY(P.t, zeros.data(), sizeof(double) * c->nch);
  INIT_COPY(P.dt, zeros.data(), sizeof(double) * c->nch);
  INIT_COPY(P.smax, zu.data(), sizeof(unsigned long long) * zu.size());
  INIT_COPY(P.n_acc, zi, 2 * sizeof(int));
  INIT_COPY(P.t + c->nch, zeros.data(), sizeof(double) * c->nch);
  if (P.fused) {
    INIT_COPY(c->n1, &n1, sizeof(int));
    INIT_COPY(c->T1.n, zi, sizeof(int) * TRI_MAX_LEVELS);
    // tag 0 is never used: the words start invalid
    if (rc == SWE_NH_OK && hipMemset(P.tw, 0, 17 * sizeof(unsigned long long) * P.ntiles) != hipSuccess)
      rc = SWE_NH_EHIP;
    INIT_COPY(P.tag1, zi, sizeof(unsigned));
    INIT_COPY(P.sweeps, zi, 2 * sizeof(int));
    INIT_COPY(P.berr, zi, 2 * sizeof(unsigned long long));
    // the one-kernel step when its blocks all fit on the device at once (block
    // 0 waits for every tile's count; the marked tiles wait for block 0)
    const bool allow = cfg->step1d_form == 0;
    P.onepass = 0;
    // (the global extension marks every tile: beyond 64 tiles its level-1
    // system would take the one-kernel form's slow path every step)
    const bool global_many = cfg->crit == SWE_NH_CRIT_GLOBAL && P.ntiles > 64;
    if (rc == SWE_NH_OK && allow && !global_many && P.ntiles <= ONEPASS_TILES) {
      const int fit = onepass_resident(P);
      P.onepass = (fit >= P.ntiles) ? 1 : 0;
    }
  }
  INIT_COPY(c->status, zi, sizeof(int));
  INIT_COPY(c->step, zi, 2 * sizeof(int));
  INIT_COPY(c->n_act, zi, sizeof(int));
  INIT_COPY(c->conv, zi, sizeof(int));
  INIT_COPY(c->iters, zi, sizeof(int));
  if (cfg->dim == 1) INIT_COPY(c->T64.n, zi, sizeof(int) * TRI_MAX_LEVELS);
  if (cfg->precision == 1 && cfg->dim == 1) INIT_COPY(c->T32.n, zi, sizeof(int) * TRI_MAX_LEVELS);
#undef INIT_COPY
  if (rc == SWE_NH_OK && cfg->dim == 2) rc = init2d(&c->cfg, &c->c2, c->k1, c->stream);
  if (rc != SWE_NH_OK) {
    (void)hipGetLastError();  // do not leave a failed call behind for the caller's next check
    swe_nh_destroy(c);
    return rc;
  }
  *out = c;
  return SWE_NH_OK;
}

void swe_nh_destroy(swe_nh_ctx* c) {
  if (!c) return;
  for (hipGraphExec_t g : {c->gexec, c->gexec2, c->gexecN, c->gexecT})
    if (g) (void)hipGraphExecDestroy(g);
  if (c->tiles_ev) (void)hipEventDestroy(c->tiles_ev);
  if (c->tiles_host) (void)hipHostFree(c->tiles_host);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

const char* swe_nh_last_error(const swe_nh_ctx* c) { return c ? c->err.c_str() : "null context"; }

int swe_nh_set_time(swe_nh_ctx* c, const double* t_host) {
  if (!c || !t_host) return SWE_NH_EINVAL;
  HIPCHK(c, hipMemcpyAsync(c->k1.t, t_host, sizeof(double) * c->nch, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SWE_NH_OK;
}

int swe_nh_get_time(swe_nh_ctx* c, double* t_host) {
  if (!c || !t_host) return SWE_NH_EINVAL;
  HIPCHK(c, hipMemcpyAsync(t_host, c->k1.t, sizeof(double) * c->nch, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SWE_NH_OK;
}

int swe_nh_step(swe_nh_ctx* c, double* h, double* hu, double* hv, double* hw, double* p,
                uint8_t* mask, int32_t nsteps) {
  if (!c || !h || !hu || !hw || !p || nsteps < 0) return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (hv == nullptr)) return fail(c, SWE_NH_EINVAL, "hv must be NULL iff dim == 1");
  const bool fused = c->cfg.dim == 1 && c->k1.fused;
  const void* key[6] = {h, hu, hv, hw, p, mask};
  bool same = c->gexec != nullptr || c->gexecT != nullptr;
  for (int i = 0; i < 6 && same; i++) same = (key[i] == c->gkey[i]);
  const bool choice = mg_choice(c);
  if (choice && c->tiles_pending) {
    // the active tiles at the end of an earlier call, if its copy is done:
    // the multigrid graph above MG_MIN_TILES of them, back to the tile
    // solver's below half of that
    const hipError_t q = hipEventQuery(c->tiles_ev);
    if (q == hipSuccess) {
      c->tiles_pending = false;
      const int nt = *c->tiles_host;
      if (nt > MG_MIN_TILES) c->mg_graph = true;
      else if (nt <= MG_MIN_TILES / 2) c->mg_graph = false;
    } else {
      (void)hipGetLastError();  // not ready is not an error of this call
    }
  }
  hipGraphExec_t* g2d = (choice && !c->mg_graph) ? &c->gexecT : &c->gexec;
  if (!same) {
    for (hipGraphExec_t* g : {&c->gexec, &c->gexec2, &c->gexecN, &c->gexecT})
      if (*g) {
        (void)hipGraphExecDestroy(*g);
        *g = nullptr;
      }
  }
  if (!same || (c->cfg.dim == 2 && *g2d == nullptr)) {
    int rc;
    if (fused) {
      // even steps: caller arrays -> workspace; odd steps: back
      rc = capture_graph(c, [&](hipStream_t s) {
        enqueue_fused1d(c, s, h, hu, hw, c->ht, c->mt, c->kt, p, mask, 0);
      }, &c->gexec);
      if (rc == SWE_NH_OK)
        rc = capture_graph(c, [&](hipStream_t s) {
          enqueue_fused1d(c, s, c->ht, c->mt, c->kt, h, hu, hw, p, mask, 1);
        }, &c->gexec2);
      // GSTEPS (even) steps per launch: the host's per-launch cost is paid
      // once for all of them; starts and ends in the caller's arrays
      if (rc == SWE_NH_OK)
        rc = capture_graph(c, [&](hipStream_t s) {
          for (int k = 0; k < GSTEPS; k += 2) {
            enqueue_fused1d(c, s, h, hu, hw, c->ht, c->mt, c->kt, p, mask, 0);
            enqueue_fused1d(c, s, c->ht, c->mt, c->kt, h, hu, hw, p, mask, 1);
          }
        }, &c->gexecN);
    } else if (c->cfg.dim == 1) {
      rc = capture_graph(c, [&](hipStream_t s) { enqueue_step1d(c, s, h, hu, hw, p, mask); },
                         &c->gexec);
    } else {
      c->c2.mg_off = g2d == &c->gexecT ? 1 : 0;
      rc = capture_graph(c, [&](hipStream_t s) {
        enqueue_step2d(&c->cfg, &c->c2, s, h, hu, hv, hw, p, mask);
      }, g2d);
      c->c2.mg_off = 0;
    }
    if (rc != SWE_NH_OK) {
      for (hipGraphExec_t* g : {&c->gexec, &c->gexec2, &c->gexecN, &c->gexecT})
        if (*g) {
          (void)hipGraphExecDestroy(*g);
          *g = nullptr;
        }
      return rc;
    }
    for (int i = 0; i < 6; i++) c->gkey[i] = key[i];
  }
  if (fused && nsteps > 0) {
    launch_speed_prologue(c->k1, h, hu, hw, c->stream);
    int rc = after_launch(c);
    if (rc) return rc;
  }
  if (c->cfg.dim == 2 && nsteps > 0) {
    launch_speed2d_prologue(&c->cfg, &c->c2, c->stream, h, hu, hv, hw);
    int rc = after_launch(c);
    if (rc) return rc;
  }
  int i = 0;
  if (fused)
    for (; i + GSTEPS <= nsteps; i += GSTEPS) HIPCHK(c, hipGraphLaunch(c->gexecN, c->stream));
  hipGraphExec_t one = c->cfg.dim == 2 ? *g2d : c->gexec;
  for (; i < nsteps; i++)
    HIPCHK(c, hipGraphLaunch((fused && (i & 1)) ? c->gexec2 : one, c->stream));
  if (choice && nsteps > 0) {
    HIPCHK(c, hipMemcpyAsync(c->tiles_host, c->c2.n_tiles_act, sizeof(int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->tiles_ev, c->stream));
    c->tiles_pending = true;
  }
  if (fused && nsteps > 0) {
    if (nsteps & 1) {  // the last step wrote the workspace copy
      launch_copy(c->ht, h, c->ncells, c->stream);
      launch_copy(c->mt, hu, c->ncells, c->stream);
      launch_copy(c->kt, hw, c->ncells, c->stream);
    }
    launch_run_end(c->k1, nsteps & 1, c->stream);
    int rc = after_launch(c);
    if (rc) return rc;
  }
  c->steps_taken += nsteps;
  return SWE_NH_OK;
}

int swe_nh_step_t(swe_nh_ctx* c, double* h, double* hu, double* hv, double* hw, double* p,
                  double* t_dev, swe_nh_stats* stats) {
  if (!c || !t_dev) return fail(c, SWE_NH_EINVAL, "bad arguments");
  const size_t tb = sizeof(double) * c->nch;
  HIPCHK(c, hipMemcpyAsync(c->k1.t, t_dev, tb, hipMemcpyDeviceToDevice, c->stream));
  int rc = swe_nh_step(c, h, hu, hv, hw, p, nullptr, 1);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(t_dev, c->k1.t, tb, hipMemcpyDeviceToDevice, c->stream));
  return stats ? swe_nh_sync_stats(c, stats) : SWE_NH_OK;
}

int swe_nh_sync_stats(swe_nh_ctx* c, swe_nh_stats* out) {
  if (!c || !out) return SWE_NH_EINVAL;
  int st = 0, na = 0, it = 0;
  double rel = 0.0, dt = 0.0, t = 0.0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int* nact = c->cfg.dim == 1 ? c->n_act : c->c2.n_act;
  HIPCHK(c, hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&na, nact, sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&it, c->cfg.dim == 1 ? c->iters : c->c2.iters, sizeof(int),
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&rel, c->cfg.dim == 1 ? c->rel : c->c2.rel, sizeof(double),
                      hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&dt, c->k1.dt, sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&t, c->k1.t, sizeof(double), hipMemcpyDeviceToHost));
  out->n_active = na;
  out->iters = it;
  out->status = status_code(st);
  out->rel_res = rel;
  out->dt = dt;
  out->t = t;
  out->steps = c->steps_taken;
  long long itsum = 0;
  if (c->cfg.dim == 2)
    HIPCHK(c, hipMemcpy(&itsum, c->c2.iters_sum, sizeof(long long), hipMemcpyDeviceToHost));
  out->iters_total = itsum;
  int z = 0;
  HIPCHK(c, hipMemcpy(c->status, &z, sizeof(int), hipMemcpyHostToDevice));
  return SWE_NH_OK;
}

int swe_nh_predict(swe_nh_ctx* c, const double* h, const double* hu, const double* hv,
                   const double* hw, const double* t_host, const double* dt_host, double* ht,
                   double* mt, double* nt, double* kt) {
  if (!c || !h || !hu || !hw || !ht || !mt || !kt || !t_host || !dt_host)
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (hv == nullptr) || (c->cfg.dim == 1) != (nt == nullptr))
    return fail(c, SWE_NH_EINVAL, "hv/nt must be NULL iff dim == 1");
  int rc = upload_stage_times(c, t_host, dt_host);
  if (rc) return rc;
  reset_status(c);
  if (c->cfg.dim == 1)
    launch_pred1d(c->k1, h, hu, hw, ht, mt, kt, c->stage_t, c->stage_dt, 0, c->stream);
  else
    launch_pred2d_stage(&c->cfg, &c->c2, c->stream, h, hu, hv, hw, c->stage_t, c->stage_dt, ht, mt,
                        nt, kt);
  return after_launch(c);
}

int swe_nh_mask(swe_nh_ctx* c, const double* ht, const double* mt, const double* nt,
                const double* kt, const double* t_host, int32_t first_step, uint8_t* mask_out,
                int64_t* n_active_host) {
  if (!c || !ht || !mt || !kt || !mask_out || !t_host) return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (nt == nullptr)) return fail(c, SWE_NH_EINVAL, "nt must be NULL iff dim == 1");
  int rc = upload_stage_times(c, t_host, nullptr);
  if (rc) return rc;
  const int mode = decide_mask_mode(&c->cfg, first_step);
  int* nact;
  if (c->cfg.dim == 1) {
    launch_mask1d(c->k1, ht, mt, kt, c->stage_t, c->stage_dt, mode, mask_out, nullptr, nullptr,
                  nullptr, nullptr, 0, c->stream);
    launch_scan(c->k1.tile_cnt, c->k1.tile_off, c->k1.ntiles, c->n_act, c->stream);
    nact = c->n_act;
  } else {
    launch_mask2d_stage(&c->cfg, &c->c2, c->stream, ht, mt, nt, kt, c->stage_t, c->stage_dt, mode,
                        mask_out);
    nact = c->c2.n_act;
  }
  rc = after_launch(c);
  if (rc) return rc;
  if (n_active_host) {
    int na = 0;
    HIPCHK(c, hipMemcpyAsync(&na, nact, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_active_host = na;
  }
  return SWE_NH_OK;
}

int swe_nh_solve_pressure(swe_nh_ctx* c, const double* ht, const double* mt, const double* nt,
                          const double* kt, const uint8_t* mask, const double* t_host,
                          const double* dt_host, double* p_inout, int32_t* iters_host,
                          double* rel_res_host) {
  if (!c || !ht || !mt || !kt || !mask || !t_host || !dt_host || !p_inout)
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (nt == nullptr)) return fail(c, SWE_NH_EINVAL, "nt must be NULL iff dim == 1");
  int rc = upload_stage_times(c, t_host, dt_host);
  if (rc) return rc;
  reset_status(c);
  hipStream_t s = c->stream;
  if (c->cfg.dim == 1) {
    K1D& P = c->k1;
    const int64_t N = c->ncells;
    launch_count1d(P, mask, s);
    launch_scan(P.tile_cnt, P.tile_off, P.ntiles, c->n_act, s);
    launch_compact1d(P, mask, s);
    launch_assemble1d(P, N, ht, mt, kt, mask, c->stage_t, c->stage_dt, c->T64.dg[0], c->T64.up[0],
                      c->T64.rh[0], s);
    solve1d(c, s, 1);
    launch_fill(p_inout, N, 0.0, s);
    launch_scatter_packed(P.act_cell, c->n_act, N, c->T64.x[0], p_inout, s);
  } else {
    solve_pressure2d(&c->cfg, &c->c2, s, ht, mt, nt, kt, mask, c->stage_t, c->stage_dt, p_inout);
  }
  rc = after_launch(c);
  if (rc) return rc;
  if (iters_host || rel_res_host) {
    int it = 0;
    double rr = 0.0;
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(&it, c->cfg.dim == 1 ? c->iters : c->c2.iters, sizeof(int),
                        hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&rr, c->cfg.dim == 1 ? c->rel : c->c2.rel, sizeof(double),
                        hipMemcpyDeviceToHost));
    if (iters_host) *iters_host = it;
    if (rel_res_host) *rel_res_host = rr;
  }
  return SWE_NH_OK;
}

int swe_nh_correct(swe_nh_ctx* c, const double* ht, const double* mt, const double* nt,
                   const double* kt, const uint8_t* mask, const double* p, const double* t_host,
                   const double* dt_host, double* m_out, double* n_out, double* k_out) {
  if (!c || !ht || !mt || !kt || !mask || !p || !t_host || !dt_host || !m_out || !k_out)
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (nt == nullptr) || (c->cfg.dim == 1) != (n_out == nullptr))
    return fail(c, SWE_NH_EINVAL, "nt/n_out must be NULL iff dim == 1");
  int rc = upload_stage_times(c, t_host, dt_host);
  if (rc) return rc;
  hipStream_t s = c->stream;
  if (c->cfg.dim == 1) {
    K1D& P = c->k1;
    const int64_t N = c->ncells;
    launch_count1d(P, mask, s);
    launch_scan(P.tile_cnt, P.tile_off, P.ntiles, c->n_act, s);
    launch_compact1d(P, mask, s);
    launch_gather_packed(P.act_cell, c->n_act, N, p, c->T64.x[0], s);
    launch_copy(mt, m_out, N, s);
    launch_copy(kt, k_out, N, s);
    launch_correct1d(P, N, ht, mt, kt, mask, c->stage_t, c->stage_dt, c->T64.x[0], m_out, k_out,
                     nullptr, s);
  } else {
    correct2d(&c->cfg, &c->c2, s, ht, mt, nt, kt, mask, p, c->stage_t, c->stage_dt, m_out, n_out,
              k_out);
  }
  return after_launch(c);
}

int swe_nh_features(swe_nh_ctx* c, const double* ht, const double* mt, const double* nt,
                    const uint8_t* mask, const double* t1_host, const double* scales_host,
                    uint16_t* out) {
  if (!c || !ht || !mt || !nt || !mask || !t1_host || !scales_host || !out)
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  for (int k = 0; k < 4; k++)
    if (!(scales_host[k] > 0.0)) return fail(c, SWE_NH_EINVAL, "feature scales must be > 0");
  if (c->cfg.dim != 2) return fail(c, SWE_NH_EINVAL, "features are defined on the 2D grid");
  int rc = upload_stage_times(c, t1_host, nullptr);
  if (rc) return rc;
  cnn_features(c->k1.ch, c->cfg.depth_static, c->cfg.nx, c->cfg.ny, c->cfg.dx, c->cfg.dy,
               scales_host, c->stage_t, c->stage_dt, ht, mt, nt, mask, out, c->stream);
  return after_launch(c);
}

int swe_nh_set_warm_start_net(swe_nh_ctx* c, const float* params, const double* scales_host,
                              double p_scale) {
  if (!c || !params || !scales_host || !(p_scale > 0.0))
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  for (int k = 0; k < 4; k++)
    if (!(scales_host[k] > 0.0)) return fail(c, SWE_NH_EINVAL, "feature scales must be > 0");
  if (c->cfg.dim != 2 || c->cfg.warm != 2)
    return fail(c, SWE_NH_EINVAL, "the network guess needs a 2D context created with warm = 2");
  c->c2.net = params;
  for (int k = 0; k < 4; k++) c->c2.fscale[k] = scales_host[k];
  c->c2.p_scale = p_scale;
  pack_net2d(&c->c2, c->stream);
  int rc = after_launch(c);
  if (rc) return rc;
  for (hipGraphExec_t* g : {&c->gexec, &c->gexec2, &c->gexecN, &c->gexecT})  // the step must pick up the network
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  return SWE_NH_OK;
}

int swe_nh_time_stage(swe_nh_ctx* c, int32_t stage, int32_t nreps, double* h, double* hu,
                      double* hv, double* hw, double* p, double* avg_us_host) {
  if (!c || !h || !hu || !hw || !p || !avg_us_host || nreps < 1 || stage < 0 || stage > 3)
    return fail(c, SWE_NH_EINVAL, "bad arguments");
  if ((c->cfg.dim == 1) != (hv == nullptr)) return fail(c, SWE_NH_EINVAL, "hv must be NULL iff dim == 1");
  if (c->cfg.dim == 1 && c->k1.fused && c->k1.onepass && (stage == 1 || stage == 2)) {
    *avg_us_host = 0.0;  // the one-kernel step has no separate level-1 solve or projection
    return SWE_NH_OK;
  }
  if (c->cfg.dim == 1 && c->k1.fused && stage == 1 && level1_local(c->k1)) {
    *avg_us_host = 0.0;  // the projection kernel solves the level-1 system itself
    return SWE_NH_OK;
  }
  // one launch of the stage, enqueued on s
  auto one = [&](hipStream_t s) {
    if (c->cfg.dim == 2) {
      time_stage2d(&c->cfg, &c->c2, s, stage, h, hu, hv, hw, p);
      return;
    }
    K1D& P = c->k1;
    uint8_t* M = c->mask_ws;
    if (P.fused) {
      // stage 0: the fused step kernel, 1: level-1 solve, 2: projection,
      // 3: the stand-alone predictor.  Outputs go to workspace scratch
      // (level-0 arrays of the packed solver, unused by this path), never
      // the caller's state; nothing advances.
      double *s0 = c->T64.dg[0], *s1 = c->T64.up[0], *s2 = c->T64.rh[0], *s3 = c->T64.x[0];
      K1D Pt = P;
      Pt.keep_speed = 1;  // replays of the step kernel must all read the same dt
      switch (stage) {
        case 0: launch_step1d(Pt, h, hu, hw, s0, s1, s2, M, s3, 0, s); break;
        case 1:
          if (level1_per_channel(P))
            launch_level1_chan(P, s);
          else
            launch_tri_solve(c->T1, c->n1, nullptr, s);
          break;
        case 2: launch_apply1d(P, M, s1, s2, s3, 0, s); break;
        default: launch_pred1d(P, h, hu, hw, c->ht, c->mt, c->kt, P.t, P.dt, 0, s);
      }
      return;
    }
    switch (stage) {
      case 0: launch_pred1d(P, h, hu, hw, c->ht, c->mt, c->kt, P.t, P.dt, 0, s); break;
      case 1: launch_mask1d(P, c->ht, c->mt, c->kt, P.t, P.dt, 0, M, nullptr, nullptr, nullptr,
                            nullptr, 0, s); break;
      case 2: solve1d(c, s, 0); break;
      default: launch_correct1d(P, c->ncells, c->ht, c->mt, c->kt, M, P.t, P.dt, c->T64.x[0],
                                hu, hw, p, s);
    }
  };
  // The launches are replayed from a graph of up to TIME_BATCH of them, so
  // that the host's per-launch cost does not enter the time of short
  // kernels; nreps is rounded up to a whole number of graph launches and
  // the mean is taken over the launches actually run.  One untimed replay
  // comes first.
  const int batch = nreps < TIME_BATCH ? nreps : TIME_BATCH;
  const int nlaunch = (nreps + batch - 1) / batch;
  hipGraphExec_t gx = nullptr;
  int rc = capture_graph(c, [&](hipStream_t s) {
    for (int r = 0; r < batch; r++) one(s);
  }, &gx);
  if (rc != SWE_NH_OK) return rc;
  hipStream_t s = c->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipGraphLaunch(gx, s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < nlaunch && e == hipSuccess; r++) e = hipGraphLaunch(gx, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(gx);
  if (e != hipSuccess) return fail(c, SWE_NH_EHIP, std::string("time_stage: ") + hipGetErrorString(e));
  *avg_us_host = 1000.0 * ms / (double(nlaunch) * batch);
  return after_launch(c);
}

}  // extern "C"

// Host runtime and C ABI of the hybrid Hermite WENO library (see include/hweno.h).
//
// A handle owns three device states for the TVD-RK3 step of eq. RK:
//   S0 = u^n, S1 = u^(1), S2 = u^(2);   stage 3 writes u^(n+1) into S0 in place (it
//   reads u^n only at the cell it updates), so a step needs no pointer rotation and a
//   captured step graph can be replayed any number of times.
// Per step, on the handle's stream (captured once into a graph and replayed; runs of eight
// steps replay a graph of eight steps, since every graph boundary idles the GPU briefly):
//   dt kernel  (Lax-Friedrichs speed of u^n -> time step, time, speed slots reset)
//   stage 1, stage 2, stage 3 (1D: one stage kernel each; 2D: flags and work lists,
//   limiter, HWENO, stage kernel; each stage also accumulates the speed of its output for
//   the next stage).
// Speeds live in four slots: slot 0 = u^n, 1 = u^(1), 2 = u^(2), 3 = u^(n+1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hweno.h"
#include "hw_dmr.h"
#include "hw_mesh1d.h"
#include "hw_stage.h"

namespace {

thread_local std::string g_last_error;

// Start of a step: the speeds of u^n (slot 3 of the previous step, or of a freshly set
// state) move to slot 0, the time step follows (fixed, or CFL), slots 1-3 are cleared.
// 1D: one thread per instance, one entry per direction.  2D (one instance): one 64-lane
// wave, lane j handling partial-maximum entry j of each direction.
__global__ void dt_kernel(int ninst, int ndir, int spread, unsigned long long* alpha, double* dt,
                          double* t, long long* steps, double fixed_dt, double T_end, double cfl,
                          const double* dxs, double dy) {
  double a[2] = {0.0, 0.0};
  int b, lane = 0, W;
  if (spread == 1) {
    b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= ninst) return;
    W = ninst * ndir;
    for (int d = 0; d < ndir; ++d) {
      const unsigned long long bits = alpha[3 * W + b * ndir + d];
      alpha[b * ndir + d] = bits;
      a[d] = __longlong_as_double((long long)bits);
    }
  } else {
    b = 0;
    lane = threadIdx.x;   // < spread <= 64
    W = ndir * spread;
    for (int d = 0; d < ndir; ++d) {
      unsigned long long bits = alpha[3 * W + d * spread + lane];
      alpha[d * spread + lane] = bits;
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long x = __shfl_xor(bits, o, 64);
        bits = x > bits ? x : bits;
      }
      a[d] = __longlong_as_double((long long)bits);
    }
  }
  double h;
  if (fixed_dt > 0.0) h = fixed_dt;
  else if (ndir == 1) h = cfl * dxs[b] / a[0];
  else h = cfl / (a[0] / dxs[b] + a[1] / dy);
  if (T_end > 0.0) {
    if (t[b] >= T_end) h = 0.0;
    else if (t[b] + h > T_end) h = T_end - t[b];
  }
  if (h > 0.0) {
    for (int s = 1; s <= 3; ++s)
      for (int d = 0; d < ndir; ++d) {
        if (spread == 1) alpha[s * W + b * ndir + d] = 0ull;
        else alpha[s * W + d * spread + lane] = 0ull;
      }
  }
  if (lane == 0) {
    dt[b] = h;
    if (h > 0.0) {
      t[b] += h;
      steps[b] += 1;
    }
  }
}

__global__ void zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

struct hw_solver {
  hw_config cfg{};
  int dim = 1, nc = 1, nmom = 2;
  long ncell = 0;               // cells per component plane
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double *S0 = nullptr, *S1 = nullptr, *S2 = nullptr, *backup = nullptr;
  uint8_t* Tn = nullptr;
  double* limn = nullptr;
  uint8_t* Hs = nullptr;                 // 2D: hybrid mask of the current stage
  uint8_t* Ts = nullptr;                 // 2D: flags of the current stage (stages 2, 3, L)
  double* lims = nullptr;                // 2D: its limited first moments (flagged cells)
  double* hwv = nullptr;                 // 2D: HWENO edge values of hybrid cells
  double* dtab = nullptr;                // double Mach reflection: prescribed ghosts of a stage
  int* wl = nullptr;                     // 2D: work lists [2 counts][flagged][hybrid]
  long long* stats = nullptr;            // 2D: list lengths of each stage of the last step [2][3]
  unsigned long long* alpha = nullptr;   // [4][aw] speed slots
  unsigned long long* alpha_op = nullptr;  // [aw]
  int aw = 1;                            // entries per slot: 1D ninst*ndir, 2D 2*ASPREAD
  double* dt = nullptr;                  // [ninst]
  double* t = nullptr;                   // [ninst]
  long long* steps = nullptr;            // [ninst]
  int* status = nullptr;
  uint8_t* flagsT[3] = {nullptr, nullptr, nullptr};
  uint8_t* flagsH[3] = {nullptr, nullptr, nullptr};
  bool export_flags = false;
  int ndir = 1;
  // 1D / batch
  int ninst = 1, maxn = 0;
  int* off = nullptr;
  double* dxs = nullptr;
  int2* items = nullptr;                 // (instance, first cell) of every tile
  int nitems = 0;
  int tile1d = 256;                      // cells per 1D tile (= threads per workgroup)
  int pgrid = 0;                         // persistent grid (0: default)
  int auto_persist = 1;                  // launch form chosen by hw_batch_tune
  std::vector<int> h_off;
  std::vector<double> h_dxs;             // per instance: the uniform cell size
  // graphs of one step and of STEPS_PER_GRAPH steps (fewer graph boundaries, each of which
  // costs the GPU several microseconds), keyed by their parameters
  hipGraphExec_t graph = nullptr;
  hipGraphExec_t graphk = nullptr;
  double graph_dt = -1.0, graph_T = -1.0;
  int graph_persist = -1, graph_grid = -1, graph_tile = -1;
  hw::Weights w{};
  // reverse mode (2D, periodic): checkpoints of the last recorded forward run, the
  // stage inputs of one segment, the segment's stage speeds, and work cotangents
  double* ckpt = nullptr;
  int adj_nck = 0, adj_k = 0, adj_nsteps = 0;
  double adj_dt = 0.0;
  bool adj_ready = false;
  double* hist = nullptr;                 // [3 adj_k + 1] states
  unsigned long long* ahist = nullptr;    // [3 adj_k + 1][2]
  double* adt = nullptr;                  // device copy of the fixed step
  double *lam = nullptr, *mu = nullptr, *G = nullptr, *acc = nullptr;
  // 2D Euler reverse: stencil, hybrid edge-value and limiter cotangents
  double *adjD = nullptr, *adjE = nullptr, *adjC = nullptr;
  // 2D Euler reverse with troubled-cell detection: every stage of the replayed segment
  // keeps what the forward's list passes computed on its input (flags, hybrid masks,
  // limited moments, HWENO edge values, work lists; [3 adj_k] stages) and its steps' list
  // lengths ([adj_k][6]), so that the reverse reads them instead of rerunning the passes
  uint8_t *recT = nullptr, *recH = nullptr;
  double *recLim = nullptr, *recHwv = nullptr;
  int* recWl = nullptr;
  long long* recStats = nullptr;
  // double Mach reflection: each recorded stage's table of prescribed ghosts ([3 adj_k]) and
  // the time of every recorded step after its dt update ([adj_ntimes]), for the replay
  double* recDtab = nullptr;
  double* adj_times = nullptr;
  int adj_ntimes = 0;
  // 1D single instance on cells of different sizes: per-cell tables (null: uniform)
  double* nu = nullptr;
  std::string err;
};

// steps per replay of the multi-step graph
constexpr int STEPS_PER_GRAPH = 8;

static hw_status fail(hw_solver* h, hw_status s, const std::string& msg) {
  if (h) h->err = msg;
  g_last_error = msg;
  return s;
}

// a failed HIP call is reported through the status; the runtime's last-error slot is
// cleared so that a later launch check does not report it again
#define HWCHK(expr)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError();                                                         \
      return fail(h, e_ == hipErrorOutOfMemory ? HW_ENOMEM : HW_EDEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    }                                                                                  \
  } while (0)

static bool weights_ok(const double* w, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!(w[i] > 0.0)) return false;
    s += w[i];
  }
  return std::fabs(s - 1.0) <= 1e-14;
}

extern "C" void hw_config_default(hw_config* c, int dim) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->dim = dim == 2 ? 2 : 1;
  c->ny = 1;
  c->x0 = 0.0;
  c->x1 = 1.0;
  c->y0 = 0.0;
  c->y1 = 1.0;
  c->eq = HW_EULER;
  c->adv[0] = 1.0;
  c->adv[1] = 1.0;
  c->gamma_gas = 1.4;
  c->bc_x = c->bc_y = HW_BC_PERIODIC;
  c->ng_edge = 3;
  c->lim_w[0] = 0.98;
  c->lim_w[1] = c->lim_w[2] = 0.01;
  if (c->dim == 1) {
    c->rec_w[0] = 0.98;
    c->rec_w[1] = c->rec_w[2] = 0.01;
  } else {
    c->rec_w[0] = 0.96;
    c->rec_w[1] = c->rec_w[2] = c->rec_w[3] = c->rec_w[4] = 0.01;
  }
  c->eps = 1e-6;
  c->cfl = 0.6;
  c->tc_mode = HW_TC_KXRCF;
  // Example 3.11: the step's corner and the Mach 3 inflow
  c->step_x = 0.6;
  c->step_y = 0.2;
  c->inflow[0] = 1.4;
  c->inflow[1] = 3.0;
  c->inflow[2] = 0.0;
  c->inflow[3] = 1.0;
}

// Forward step: the cell indices (si, sj) of the step's corner (solid cells gx >= si,
// gy < sj) and the conserved inflow state; any other boundary: si = nx, sj = 0 (no solid
// cell).  ok: whether the corner lies on cell faces.
static bool step_geometry(const hw_config* c, int* si, int* sj, double* uin) {
  *si = c->nx;
  *sj = 0;
  for (int i = 0; i < 4; ++i) uin[i] = 0.0;
  if (c->bc_x != HW_BC_STEP) return true;
  const double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
  const double a = (c->step_x - c->x0) / dx, b = (c->step_y - c->y0) / dy;
  if (!std::isfinite(a) || !std::isfinite(b) || std::fabs(a) > 1e9 || std::fabs(b) > 1e9) return false;
  *si = (int)std::lround(a);
  *sj = (int)std::lround(b);
  const double rho = c->inflow[0], u = c->inflow[1], v = c->inflow[2], p = c->inflow[3];
  uin[0] = rho;
  uin[1] = rho * u;
  uin[2] = rho * v;
  uin[3] = p / (c->gamma_gas - 1.0) + 0.5 * rho * (u * u + v * v);
  return std::fabs(a - *si) <= 1e-9 && std::fabs(b - *sj) <= 1e-9;
}

static hw_status validate(const hw_config* c, std::string& msg) {
  if (c->dim != 1 && c->dim != 2) { msg = "dim must be 1 or 2"; return HW_EINVAL; }
  if (c->eq < 0 || c->eq > 2) { msg = "unknown equation"; return HW_EINVAL; }
  if (c->nx < 7 || (c->dim == 2 && c->ny < 7)) { msg = "need at least 7 cells per direction"; return HW_EINVAL; }
  if (!(c->x1 > c->x0) || (c->dim == 2 && !(c->y1 > c->y0))) { msg = "empty domain"; return HW_EINVAL; }
  if (c->bc_x < 0 || c->bc_x > 4 || c->bc_y < 0 || c->bc_y > 4) { msg = "unknown boundary condition"; return HW_EINVAL; }
  if (c->bc_x == HW_BC_STEP || c->bc_y == HW_BC_STEP) {
    if (c->dim != 2 || c->eq != HW_EULER || c->bc_x != HW_BC_STEP || c->bc_y != HW_BC_STEP) {
      msg = "the forward-step boundaries apply to 2D Euler, on all four sides (bc_x = bc_y)";
      return HW_EINVAL;
    }
    int si, sj;
    double uin[4];
    if (!step_geometry(c, &si, &sj, uin)) { msg = "the step's corner must lie on cell faces"; return HW_EINVAL; }
    if (sj < 3 || 2 * sj > c->ny || si < sj || si > c->nx - 1) {
      msg = "the step's corner cells (si, sj) need 3 <= sj, 2 sj <= ny and sj <= si < nx";
      return HW_EINVAL;
    }
    if (!(c->inflow[0] > 0.0) || !(c->inflow[3] > 0.0) || !std::isfinite(c->inflow[1]) ||
        !std::isfinite(c->inflow[2])) {
      msg = "the inflow state needs rho > 0, p > 0 and finite velocities";
      return HW_EINVAL;
    }
  }
  if (c->bc_x == HW_BC_DMR || c->bc_y == HW_BC_DMR) {
    if (c->dim != 2 || c->eq != HW_EULER || c->bc_x != HW_BC_DMR || c->bc_y != HW_BC_DMR) {
      msg = "the double Mach reflection boundaries apply to 2D Euler, on all four sides (bc_x = bc_y)";
      return HW_EINVAL;
    }
  }
  if ((c->bc_x == HW_BC_REFLECTIVE || (c->dim == 2 && c->bc_y == HW_BC_REFLECTIVE)) && c->eq != HW_EULER) {
    msg = "reflective walls are defined for the Euler equations";
    return HW_EINVAL;
  }
  if (c->tc_mode < 0 || c->tc_mode > 2) { msg = "unknown troubled-cell mode"; return HW_EINVAL; }
  if (c->dim == 2 && c->ng_edge != 2 && c->ng_edge != 3) { msg = "ng_edge must be 2 or 3"; return HW_EINVAL; }
  if (!weights_ok(c->lim_w, 3)) { msg = "limiter linear weights must be positive and sum to 1"; return HW_EINVAL; }
  if (!weights_ok(c->rec_w, c->dim == 1 ? 3 : 5)) { msg = "reconstruction linear weights must be positive and sum to 1"; return HW_EINVAL; }
  if (!(c->eps > 0.0)) { msg = "eps must be positive"; return HW_EINVAL; }
  if (!(c->cfl > 0.0)) { msg = "cfl must be positive"; return HW_EINVAL; }
  if (c->eq == HW_EULER && !(c->gamma_gas > 1.0)) { msg = "gamma_gas must exceed 1"; return HW_EINVAL; }
  if (c->dim == 2) {
    const double dx = (c->x1 - c->x0) / c->nx, dy = (c->y1 - c->y0) / c->ny;
    if (std::fabs(dx - dy) > 1e-12 * dx) { msg = "2D cells must be square"; return HW_EINVAL; }
    if ((double)c->nx * c->ny > 2.0e9) { msg = "mesh too large"; return HW_EINVAL; }
  }
  return HW_OK;
}

static void set_weights(hw_solver* h) {
  for (int i = 0; i < 3; ++i) h->w.lim[i] = h->cfg.lim_w[i];
  for (int i = 0; i < 5; ++i) h->w.rec[i] = h->cfg.rec_w[i];
  h->w.eps = h->cfg.eps;
}

static hw_status alloc_common(hw_solver* h) {
  const size_t st = (size_t)h->nmom * h->nc * h->ncell * sizeof(double);
  HWCHK(hipMalloc(&h->S0, st));
  HWCHK(hipMalloc(&h->S1, st));
  HWCHK(hipMalloc(&h->S2, st));
  HWCHK(hipMalloc(&h->backup, st));
  HWCHK(hipMalloc(&h->Tn, h->ncell));
  HWCHK(hipMalloc(&h->limn, (size_t)(h->nmom - 1) * h->nc * h->ncell * sizeof(double)));
  if (h->dim == 2 && h->cfg.tc_mode != HW_TC_NONE) {
    HWCHK(hipMalloc(&h->Ts, h->ncell));
    HWCHK(hipMalloc(&h->Hs, h->ncell));
    HWCHK(hipMalloc(&h->lims, (size_t)(h->nmom - 1) * h->nc * h->ncell * sizeof(double)));
    HWCHK(hipMalloc(&h->hwv, (size_t)4 * h->cfg.ng_edge * h->nc * h->ncell * sizeof(double)));
    HWCHK(hipMalloc(&h->wl, (2 + 2 * (size_t)h->ncell) * sizeof(int)));
    HWCHK(hipMemsetAsync(h->wl, 0, 2 * sizeof(int), h->stream));
    HWCHK(hipMalloc(&h->stats, 6 * sizeof(long long)));
    HWCHK(hipMemsetAsync(h->stats, 0, 6 * sizeof(long long), h->stream));
  }
  if (h->cfg.bc_x == HW_BC_DMR)
    HWCHK(hipMalloc(&h->dtab, (size_t)12 * (4 * (h->cfg.nx + 4) + 4 * h->cfg.ny) * sizeof(double)));
  h->aw = h->dim == 2 ? 2 * hw::ASPREAD : h->ninst * h->ndir;
  const int W = h->aw;
  HWCHK(hipMalloc(&h->alpha, 4 * W * sizeof(unsigned long long)));
  HWCHK(hipMalloc(&h->alpha_op, W * sizeof(unsigned long long)));
  HWCHK(hipMalloc(&h->dt, h->ninst * sizeof(double)));
  HWCHK(hipMalloc(&h->t, h->ninst * sizeof(double)));
  HWCHK(hipMalloc(&h->steps, h->ninst * sizeof(long long)));
  HWCHK(hipMalloc(&h->status, sizeof(int)));
  HWCHK(hipMemsetAsync(h->S0, 0, st, h->stream));
  HWCHK(hipMemsetAsync(h->Tn, 0, h->ncell, h->stream));
  HWCHK(hipMemsetAsync(h->alpha, 0, 4 * W * sizeof(unsigned long long), h->stream));
  HWCHK(hipMemsetAsync(h->t, 0, h->ninst * sizeof(double), h->stream));
  HWCHK(hipMemsetAsync(h->steps, 0, h->ninst * sizeof(long long), h->stream));
  HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
  return HW_OK;
}

static hw_status build_items(hw_solver* h, int tile) {
  std::vector<int2> items;
  for (int b = 0; b < h->ninst; ++b)
    for (int i0 = 0; i0 < h->h_off[b + 1] - h->h_off[b]; i0 += tile) items.push_back(make_int2(b, i0));
  if (h->items) HWCHK(hipFree(h->items));
  h->items = nullptr;
  h->nitems = 0;
  HWCHK(hipMalloc(&h->items, items.size() * sizeof(int2)));
  HWCHK(hipMemcpy(h->items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
  h->nitems = (int)items.size();
  h->tile1d = tile;
  return HW_OK;
}

static hw_status setup_1d(hw_solver* h, const std::vector<int>& nxs, const std::vector<double>& dxs) {
  h->ninst = (int)nxs.size();
  h->h_off.assign(h->ninst + 1, 0);
  h->maxn = 0;
  for (int b = 0; b < h->ninst; ++b) {
    h->h_off[b + 1] = h->h_off[b] + nxs[b];
    h->maxn = std::max(h->maxn, nxs[b]);
  }
  h->ncell = h->h_off[h->ninst];
  h->h_dxs = dxs;
  HWCHK(hipMalloc(&h->off, (h->ninst + 1) * sizeof(int)));
  HWCHK(hipMalloc(&h->dxs, h->ninst * sizeof(double)));
  HWCHK(hipMemcpyAsync(h->off, h->h_off.data(), (h->ninst + 1) * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipMemcpyAsync(h->dxs, dxs.data(), h->ninst * sizeof(double), hipMemcpyHostToDevice, h->stream));
  hw_status s = build_items(h, 256);
  if (s != HW_OK) return s;
  return alloc_common(h);
}

static hw_status make_stream(hw_solver* h, void* stream) {
  if (stream) {
    h->stream = (hipStream_t)stream;
    h->own_stream = false;
  } else {
    HWCHK(hipStreamCreate(&h->stream));
    h->own_stream = true;
  }
  return HW_OK;
}

extern "C" hw_status hw_create(const hw_config* cfg, void* stream, hw_solver** out) {
  hw_solver* h = nullptr;
  if (!cfg || !out) return fail(nullptr, HW_EINVAL, "null argument");
  std::string msg;
  if (validate(cfg, msg) != HW_OK) return fail(nullptr, HW_EINVAL, msg);
  h = new hw_solver();
  h->cfg = *cfg;
  if (h->cfg.dim == 1) h->cfg.ny = 1;
  h->dim = cfg->dim;
  h->nc = cfg->eq == HW_EULER ? cfg->dim + 2 : 1;
  h->nmom = cfg->dim + 1;
  h->ndir = cfg->dim;
  set_weights(h);
  hw_status s = make_stream(h, stream);
  if (s == HW_OK) {
    if (cfg->dim == 1) {
      s = setup_1d(h, {cfg->nx}, {(cfg->x1 - cfg->x0) / cfg->nx});
    } else {
      h->ncell = (long)cfg->nx * cfg->ny;
      const double dx = (cfg->x1 - cfg->x0) / cfg->nx;
      hipError_t e = hipMalloc(&h->dxs, sizeof(double));
      if (e != hipSuccess) s = fail(h, HW_ENOMEM, "hipMalloc dx");
      else e = hipMemcpy(h->dxs, &dx, sizeof(double), hipMemcpyHostToDevice);
      if (s == HW_OK && e != hipSuccess) s = fail(h, HW_EDEVICE, hipGetErrorString(e));
      if (s == HW_OK) s = alloc_common(h);
    }
  }
  if (s != HW_OK) {
    std::string m = h->err;
    hw_destroy(h);
    return fail(nullptr, s, m);
  }
  *out = h;
  return HW_OK;
}

extern "C" hw_status hw_batch_create(const hw_config* base, int n, const int* nx, const double* x0,
                                     const double* x1, void* stream, hw_solver** out) {
  if (!base || !nx || !out || n <= 0) return fail(nullptr, HW_EINVAL, "invalid batch arguments");
  if (base->dim != 1) return fail(nullptr, HW_EINVAL, "batches are one-dimensional");
  std::vector<int> nxs(n);
  std::vector<double> dxs(n);
  long total = 0;
  for (int b = 0; b < n; ++b) {
    hw_config c = *base;
    c.nx = nx[b];
    if (x0) c.x0 = x0[b];
    if (x1) c.x1 = x1[b];
    std::string msg;
    if (validate(&c, msg) != HW_OK) return fail(nullptr, HW_EINVAL, "instance " + std::to_string(b) + ": " + msg);
    nxs[b] = nx[b];
    dxs[b] = (c.x1 - c.x0) / c.nx;
    total += nx[b];
  }
  if (total > 2000000000L) return fail(nullptr, HW_EINVAL, "batch too large");
  hw_solver* h = new hw_solver();
  h->cfg = *base;
  h->cfg.ny = 1;
  h->dim = 1;
  h->nc = base->eq == HW_EULER ? 3 : 1;
  h->nmom = 2;
  h->ndir = 1;
  set_weights(h);
  hw_status s = make_stream(h, stream);
  if (s == HW_OK) s = setup_1d(h, nxs, dxs);
  if (s != HW_OK) {
    std::string m = h->err;
    hw_destroy(h);
    return fail(nullptr, s, m);
  }
  *out = h;
  return HW_OK;
}

extern "C" hw_status hw_destroy(hw_solver* h) {
  if (!h) return HW_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->graphk) (void)hipGraphExecDestroy(h->graphk);
  void* ptrs[] = {h->S0, h->S1, h->S2, h->backup, h->Tn, h->limn, h->Ts, h->Hs, h->lims, h->hwv, h->wl, h->stats,
                  h->alpha, h->alpha_op, h->dt,
                  h->t, h->steps, h->status, h->off, h->dxs, h->items,
                  h->flagsT[0], h->flagsT[1], h->flagsT[2], h->flagsH[0], h->flagsH[1], h->flagsH[2],
                  h->ckpt, h->hist, h->ahist, h->adt, h->lam, h->mu, h->G, h->acc,
                  h->adjD, h->adjE, h->adjC, h->nu, h->dtab,
                  h->recT, h->recH, h->recLim, h->recHwv, h->recWl, h->recStats, h->recDtab,
                  h->adj_times};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return HW_OK;
}

extern "C" hw_status hw_get_sizes(const hw_solver* h, long* cells, int* ncomp, int* nmoments) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (cells) *cells = h->ncell;
  if (ncomp) *ncomp = h->nc;
  if (nmoments) *nmoments = h->nmom;
  return HW_OK;
}

// ------------------------------------------------------------------------------ launches

static hw_status launch_alpha(hw_solver* h, const double* U, unsigned long long* out) {
  const int W = h->aw;
  hipLaunchKernelGGL(zero_u64, dim3((W + 255) / 256), dim3(256), 0, h->stream, out, W);
  HWCHK(hipGetLastError());
  if (h->dim == 2) {
    int si, sj;
    double uin[4];
    step_geometry(&h->cfg, &si, &sj, uin);
    HWCHK(hw_launch_alpha2d(h->cfg.eq, U, h->cfg.nx, h->cfg.ny, h->cfg.gamma_gas, h->cfg.adv[0],
                            h->cfg.adv[1], si, sj, out, h->stream));
  }
  else
    HWCHK(hw_launch_alpha1d(h->cfg.eq, U, h->off, h->ninst, (int)h->ncell, h->maxn,
                            h->cfg.gamma_gas, h->cfg.adv[0], out, h->stream));
  return HW_OK;
}

// Where one 2D stage keeps its list passes' results: flags T, hybrid masks H, limited
// moments, HWENO edge values, work lists (counts, flagged, hybrid) and the step's list
// lengths; Tn / limn: those of the step's first stage (u^n), read by its second and third.
struct StageRec {
  uint8_t *T, *H, *Tn;
  double *lim, *hwv, *limn;
  int* wl;
  long long* stats;
  int st;             // stage of the step (0, 1, 2)
  double* dtab;       // double Mach reflection: the stage's prescribed ghosts (else null)
  const double* t;    // double Mach reflection: the step's time after its dt update (else null)
};

// slot r = 3 i + stage of the recorded segment (step i)
static StageRec stage_rec(hw_solver* h, int r) {
  const size_t n = h->ncell;
  const size_t nl = (size_t)(h->nmom - 1) * h->nc * n, nh = (size_t)4 * h->cfg.ng_edge * h->nc * n;
  const int r0 = r - r % 3;
  StageRec q;
  q.T = h->recT + (size_t)r * n;
  q.H = h->recH + (size_t)r * n;
  q.Tn = h->recT + (size_t)r0 * n;
  q.lim = h->recLim + (size_t)r * nl;
  q.limn = h->recLim + (size_t)r0 * nl;
  q.hwv = h->recHwv + (size_t)r * nh;
  q.wl = h->recWl + (size_t)r * (2 + 2 * n);
  q.stats = h->recStats + (size_t)(r / 3) * 6;
  q.st = r % 3;
  q.dtab = h->recDtab ? h->recDtab + (size_t)r * 12 * hw::dmr::ring2_size(h->cfg.nx, h->cfg.ny) : nullptr;
  q.t = nullptr;
  return q;
}

static hw_status launch_stage(hw_solver* h, int mode, const double* in, const double* base,
                              double* out, const unsigned long long* ain, unsigned long long* aout,
                              int fslot, double* wout, int persistent,
                              const double* dtp = nullptr, hipEvent_t* ev = nullptr,
                              const StageRec* rec = nullptr) {
  uint8_t* fT = (h->export_flags && fslot >= 0) ? h->flagsT[fslot] : nullptr;
  uint8_t* fH = (h->export_flags && fslot >= 0) ? h->flagsH[fslot] : nullptr;
  if (h->dim == 2) {
    hw::Stage2D P{};
    P.in = in; P.base = base; P.out = out; P.Tn = h->Tn; P.limn = h->limn;
    P.Tcur = mode == hw::MODE_RK1 ? h->Tn : h->Ts;
    P.limcur = mode == hw::MODE_RK1 ? h->limn : h->lims;
    P.Hcur = h->Hs;
    P.G = h->hwv;
    if (h->wl) {
      P.counts = h->wl;
      P.flist = h->wl + 2;
      P.hlist = h->wl + 2 + h->ncell;
      P.stats = h->stats;
    }
    if (rec) {   // a stage of a recorded segment: its list passes' results kept in rec
      P.Tn = rec->Tn; P.limn = rec->limn;
      P.Tcur = rec->T; P.limcur = rec->lim; P.Hcur = rec->H; P.G = rec->hwv;
      P.counts = rec->wl;
      P.flist = rec->wl + 2;
      P.hlist = rec->wl + 2 + h->ncell;
      P.stats = rec->stats;
    }
    P.alpha_in = ain; P.alpha_out = aout; P.dt = dtp ? dtp : h->dt;
    P.flagsT = fT; P.flagsH = fH; P.wout = wout; P.status = h->status;
    P.nx = h->cfg.nx; P.ny = h->cfg.ny; P.bcx = h->cfg.bc_x; P.bcy = h->cfg.bc_y;
    P.tc_mode = h->cfg.tc_mode; P.mode = mode;
    P.dx = (h->cfg.x1 - h->cfg.x0) / h->cfg.nx;
    P.dy = (h->cfg.y1 - h->cfg.y0) / h->cfg.ny;
    P.h = 0.5 * std::sqrt(P.dx * P.dx + P.dy * P.dy);
    P.idx = 1.0 / P.dx;
    P.idy = 1.0 / P.dy;
    P.gam = h->cfg.gamma_gas; P.adv0 = h->cfg.adv[0]; P.adv1 = h->cfg.adv[1];
    P.x0 = h->cfg.x0; P.y0 = h->cfg.y0; P.t = h->t; P.dtab = h->dtab;
    if (rec && rec->dtab) P.dtab = rec->dtab;   // the recorded stage's own table
    if (rec && rec->t) P.t = rec->t;            // and its step's time
    step_geometry(&h->cfg, &P.si, &P.sj, P.uin);
    P.w = h->w;
    HWCHK(hw_launch_stage2d(h->cfg.eq, h->cfg.ng_edge, &P, h->stream, ev));
  } else {
    hw::Stage1D P{};
    P.in = in; P.base = base; P.out = out; P.Tn = h->Tn; P.limn = h->limn;
    P.items = h->items; P.off = h->off; P.dxs = h->dxs;
    P.alpha_in = ain; P.alpha_out = aout; P.dt = h->dt;
    P.flagsT = fT; P.flagsH = fH; P.wout = wout; P.status = h->status;
    P.nitems = h->nitems; P.total = (int)h->ncell; P.bc = h->cfg.bc_x;
    P.tc_mode = h->cfg.tc_mode; P.mode = mode;
    P.gam = h->cfg.gamma_gas; P.adv = h->cfg.adv[0];
    P.w = h->w;
    P.nu = h->nu;
    int grid = h->pgrid > 0 ? h->pgrid : 1024;
    HWCHK(hw_launch_stage1d(h->cfg.eq, persistent, grid, h->tile1d, &P, h->stream));
  }
  return HW_OK;
}

// enqueue one step (dt kernel + three stages); fixed_dt > 0 fixes dt, T_end > 0 clips
static void launch_dt(hw_solver* h, double fixed_dt, double T_end) {
  const double dy = h->dim == 2 ? (h->cfg.y1 - h->cfg.y0) / h->cfg.ny : 1.0;
  if (h->dim == 2)
    hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(64), 0, h->stream, 1, 2, hw::ASPREAD, h->alpha, h->dt,
                       h->t, h->steps, fixed_dt, T_end, h->cfg.cfl, h->dxs, dy);
  else
    hipLaunchKernelGGL(dt_kernel, dim3((h->ninst + 63) / 64), dim3(64), 0, h->stream, h->ninst, h->ndir, 1,
                       h->alpha, h->dt, h->t, h->steps, fixed_dt, T_end, h->cfg.cfl, h->dxs, dy);
}

static hw_status enqueue_step(hw_solver* h, double fixed_dt, double T_end, int persistent) {
  const int W = h->aw;
  launch_dt(h, fixed_dt, T_end);
  HWCHK(hipGetLastError());
  hw_status s;
  if ((s = launch_stage(h, hw::MODE_RK1, h->S0, h->S0, h->S1, h->alpha, h->alpha + W, 0, nullptr, persistent)) != HW_OK) return s;
  if ((s = launch_stage(h, hw::MODE_RK2, h->S1, h->S0, h->S2, h->alpha + W, h->alpha + 2 * W, 1, nullptr, persistent)) != HW_OK) return s;
  if ((s = launch_stage(h, hw::MODE_RK3, h->S2, h->S0, h->S0, h->alpha + 2 * W, h->alpha + 3 * W, 2, nullptr, persistent)) != HW_OK) return s;
  return HW_OK;
}

static hw_status sync(hw_solver* h) {
  HWCHK(hipStreamSynchronize(h->stream));
  return HW_OK;
}

static hw_status read_status(hw_solver* h, int* st) {
  HWCHK(hipMemcpyAsync(st, h->status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  return HW_OK;
}

static hw_status after_state_change(hw_solver* h) {
  // speed of the new state into slot 3 (read by the next step's dt kernel), time 0
  const int W = h->aw;
  hw_status s = launch_alpha(h, h->S0, h->alpha + 3 * W);
  if (s != HW_OK) return s;
  HWCHK(hipMemsetAsync(h->t, 0, h->ninst * sizeof(double), h->stream));
  HWCHK(hipMemsetAsync(h->steps, 0, h->ninst * sizeof(long long), h->stream));
  HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
  return sync(h);
}

extern "C" hw_status hw_set_state(hw_solver* h, const double* avg, const double* mx, const double* my) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!avg || !mx || (h->dim == 2 && !my)) return fail(h, HW_EINVAL, "null state array");
  const size_t plane = (size_t)h->nc * h->ncell;
  const double* src[3] = {avg, mx, my};
  for (int m = 0; m < h->nmom; ++m)
    HWCHK(hipMemcpyAsync(h->S0 + m * plane, src[m], plane * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return after_state_change(h);
}

extern "C" hw_status hw_set_state_device(hw_solver* h, const double* d) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!d) return fail(h, HW_EINVAL, "null state array");
  const size_t n = (size_t)h->nmom * h->nc * h->ncell;
  HWCHK(hipMemcpyAsync(h->S0, d, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return after_state_change(h);
}

extern "C" hw_status hw_get_state(hw_solver* h, double* avg, double* mx, double* my, double* t) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  const size_t plane = (size_t)h->nc * h->ncell;
  double* dst[3] = {avg, mx, my};
  for (int m = 0; m < h->nmom; ++m)
    if (dst[m]) HWCHK(hipMemcpyAsync(dst[m], h->S0 + m * plane, plane * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (t) HWCHK(hipMemcpyAsync(t, h->t, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  return sync(h);
}

extern "C" hw_status hw_get_state_device(hw_solver* h, double* d) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!d) return fail(h, HW_EINVAL, "null state array");
  const size_t n = (size_t)h->nmom * h->nc * h->ncell;
  HWCHK(hipMemcpyAsync(d, h->S0, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return HW_OK;
}

static hw_status ensure_flags(hw_solver* h) {
  for (int s = 0; s < 3; ++s) {
    if (!h->flagsT[s]) HWCHK(hipMalloc(&h->flagsT[s], h->ncell));
    if (!h->flagsH[s]) HWCHK(hipMalloc(&h->flagsH[s], h->ncell));
  }
  return HW_OK;
}

static void drop_graph(hw_solver* h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->graphk) (void)hipGraphExecDestroy(h->graphk);
  h->graph = nullptr;
  h->graphk = nullptr;
  h->graph_dt = h->graph_T = -1.0;
  h->graph_persist = h->graph_grid = h->graph_tile = -1;
}

extern "C" hw_status hw_set_flag_export(hw_solver* h, int on) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (on) {
    hw_status s = ensure_flags(h);
    if (s != HW_OK) return s;
  }
  h->export_flags = on != 0;
  drop_graph(h);
  return HW_OK;
}

extern "C" hw_status hw_get_flags(hw_solver* h, int stage, unsigned char* T, unsigned char* H) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (stage < 0 || stage > 2) return fail(h, HW_EINVAL, "stage must be 0, 1 or 2");
  if (!h->flagsT[stage]) return fail(h, HW_ESTATE, "flag export is off");
  if (T) HWCHK(hipMemcpyAsync(T, h->flagsT[stage], h->ncell, hipMemcpyDeviceToHost, h->stream));
  if (H) HWCHK(hipMemcpyAsync(H, h->flagsH[stage], h->ncell, hipMemcpyDeviceToHost, h->stream));
  return sync(h);
}

extern "C" hw_status hw_get_stats(hw_solver* h, double* alpha, long* flagged, long* hybrid) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (alpha) {
    // speeds of the current state: slot 3, maximum over its entries per direction
    const int W = h->aw;
    std::vector<unsigned long long> a(W);
    HWCHK(hipMemcpyAsync(a.data(), h->alpha + 3 * W, W * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         h->stream));
    hw_status s = sync(h);
    if (s != HW_OK) return s;
    for (int d = 0; d < h->ndir; ++d) {
      unsigned long long m = 0;
      for (int j = 0; j < W; ++j) {
        const int dj = h->dim == 2 ? j / hw::ASPREAD : j % h->ndir;
        if (dj == d) m = std::max(m, a[j]);
      }
      double v;
      std::memcpy(&v, &m, sizeof v);
      alpha[d] = v;
    }
  }
  if (flagged || hybrid) {
    long f[3] = {-1, -1, -1}, hy[3] = {-1, -1, -1};
    if (h->dim == 2 && h->stats) {
      long long c[6];
      HWCHK(hipMemcpyAsync(c, h->stats, sizeof c, hipMemcpyDeviceToHost, h->stream));
      hw_status s = sync(h);
      if (s != HW_OK) return s;
      for (int k = 0; k < 3; ++k) { f[k] = (long)c[k]; hy[k] = (long)c[3 + k]; }
    } else if (h->dim == 2 || h->cfg.tc_mode == HW_TC_NONE) {
      for (int k = 0; k < 3; ++k) f[k] = hy[k] = 0;
    } else if (h->flagsT[0]) {
      // 1D: counted from the exported flags
      std::vector<unsigned char> T(h->ncell), H(h->ncell);
      for (int k = 0; k < 3; ++k) {
        HWCHK(hipMemcpyAsync(T.data(), h->flagsT[k], h->ncell, hipMemcpyDeviceToHost, h->stream));
        HWCHK(hipMemcpyAsync(H.data(), h->flagsH[k], h->ncell, hipMemcpyDeviceToHost, h->stream));
        hw_status s = sync(h);
        if (s != HW_OK) return s;
        long a = 0, b = 0;
        for (long i = 0; i < h->ncell; ++i) { a += T[i] != 0; b += H[i] != 0; }
        f[k] = a;
        hy[k] = b;
      }
    }
    for (int k = 0; k < 3; ++k) {
      if (flagged) flagged[k] = f[k];
      if (hybrid) hybrid[k] = hy[k];
    }
  }
  return HW_OK;
}

extern "C" hw_status hw_set_linear_weights(hw_solver* h, const double* lim_w, const double* rec_w) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (lim_w) {
    if (!weights_ok(lim_w, 3)) return fail(h, HW_EINVAL, "limiter linear weights must be positive and sum to 1");
    for (int i = 0; i < 3; ++i) h->cfg.lim_w[i] = lim_w[i];
  }
  if (rec_w) {
    const int n = h->dim == 1 ? 3 : 5;
    if (!weights_ok(rec_w, n)) return fail(h, HW_EINVAL, "reconstruction linear weights must be positive and sum to 1");
    for (int i = 0; i < n; ++i) h->cfg.rec_w[i] = rec_w[i];
  }
  set_weights(h);
  drop_graph(h);
  return HW_OK;
}

extern "C" hw_status hw_step(hw_solver* h, double dt) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!std::isfinite(dt)) return fail(h, HW_EINVAL, "dt must be finite");
  const size_t n = (size_t)h->nmom * h->nc * h->ncell;
  const int W = h->aw;
  std::vector<unsigned long long> asave(W);
  std::vector<double> tsave(h->ninst);
  std::vector<long long> ssave(h->ninst);
  HWCHK(hipMemcpyAsync(h->backup, h->S0, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HWCHK(hipMemcpyAsync(asave.data(), h->alpha + 3 * W, W * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipMemcpyAsync(tsave.data(), h->t, h->ninst * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipMemcpyAsync(ssave.data(), h->steps, h->ninst * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
  hw_status s = enqueue_step(h, dt > 0.0 ? dt : 0.0, 0.0, 0);
  if (s != HW_OK) return s;
  int st = 0;
  if ((s = read_status(h, &st)) != HW_OK) return s;
  if (st) {
    HWCHK(hipMemcpyAsync(h->S0, h->backup, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HWCHK(hipMemcpyAsync(h->alpha + 3 * W, asave.data(), W * sizeof(unsigned long long), hipMemcpyHostToDevice, h->stream));
    HWCHK(hipMemcpyAsync(h->t, tsave.data(), h->ninst * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HWCHK(hipMemcpyAsync(h->steps, ssave.data(), h->ninst * sizeof(long long), hipMemcpyHostToDevice, h->stream));
    HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
    (void)sync(h);
    return fail(h, HW_ENONFINITE, (st & 2) ? "non-physical state (rho <= 0 or p <= 0)" : "non-finite value");
  }
  return HW_OK;
}

static hw_status capture_step(hw_solver* h, double fixed_dt, double T_end, int persistent,
                              long nsteps);

// n steps from the captured graphs: STEPS_PER_GRAPH at a time, then one at a time
static hw_status launch_steps(hw_solver* h, long n) {
  for (; n >= STEPS_PER_GRAPH; n -= STEPS_PER_GRAPH) HWCHK(hipGraphLaunch(h->graphk, h->stream));
  for (; n > 0; --n) HWCHK(hipGraphLaunch(h->graph, h->stream));
  return HW_OK;
}

// steps are replayed from one captured graph of the step's launches (the step reads dt,
// speeds and work-list counts from device memory, so every replay is the same launch set)
extern "C" hw_status hw_steps(hw_solver* h, int nsteps, double dt) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(h, HW_EINVAL, "invalid step count or dt");
  if (nsteps == 0) return HW_OK;
  hw_status s = capture_step(h, dt > 0.0 ? dt : 0.0, 0.0, 0, nsteps);
  if (s != HW_OK) return s;
  return launch_steps(h, nsteps);
}

extern "C" hw_status hw_run(hw_solver* h, double T, long max_steps, long* steps_out, double* t_out) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!(T > 0.0) || !std::isfinite(T) || max_steps < 0) return fail(h, HW_EINVAL, "invalid final time or step limit");
  std::vector<double> tt(h->ninst);
  std::vector<long long> ss(h->ninst);
  HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
  long long start = 0;
  HWCHK(hipMemcpyAsync(&start, h->steps, sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  long done_steps = 0;
  while (true) {
    const long chunk = std::min<long>(16, max_steps - done_steps);
    if (chunk <= 0) break;
    hw_status s = capture_step(h, 0.0, T, 0, chunk);
    if (s != HW_OK) return s;
    if ((s = launch_steps(h, chunk)) != HW_OK) return s;
    HWCHK(hipMemcpyAsync(tt.data(), h->t, h->ninst * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HWCHK(hipMemcpyAsync(ss.data(), h->steps, h->ninst * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
    int st = 0;
    if ((s = read_status(h, &st)) != HW_OK) return s;
    done_steps = (long)(*std::max_element(ss.begin(), ss.end()) - start);
    if (st) {
      if (steps_out) *steps_out = done_steps;
      if (t_out) *t_out = tt[0];
      return fail(h, HW_ENONFINITE, (st & 2) ? "non-physical state (rho <= 0 or p <= 0)" : "non-finite value");
    }
    if (*std::min_element(tt.begin(), tt.end()) >= T) break;
  }
  if (steps_out) *steps_out = done_steps;
  if (t_out) *t_out = tt[0];
  return HW_OK;
}

extern "C" hw_status hw_apply_operator(hw_solver* h, const double* d_in, double* d_L, double* d_lim) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!d_in || !d_L) return fail(h, HW_EINVAL, "null device array");
  hw_status s = launch_alpha(h, d_in, h->alpha_op);
  if (s != HW_OK) return s;
  return launch_stage(h, hw::MODE_L, d_in, d_in, d_L, h->alpha_op, nullptr, 0, d_lim, 0);
}

extern "C" hw_status hw_set_time(hw_solver* h, double t) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!std::isfinite(t) || t < 0.0) return fail(h, HW_EINVAL, "the time must be finite and non-negative");
  std::vector<double> tt(h->ninst, t);
  HWCHK(hipMemcpyAsync(h->t, tt.data(), h->ninst * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return sync(h);
}

extern "C" hw_status hw_get_time(hw_solver* h, double* times, long* steps) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  std::vector<long long> ss(h->ninst);
  if (times) HWCHK(hipMemcpyAsync(times, h->t, h->ninst * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipMemcpyAsync(ss.data(), h->steps, h->ninst * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  if (steps) *steps = (long)*std::max_element(ss.begin(), ss.end());
  return HW_OK;
}

extern "C" hw_status hw_profile_steps(hw_solver* h, int nsteps, double dt, double* ms_stage,
                                     double* ms_step, double* ms_kernels) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (nsteps <= 0) return fail(h, HW_EINVAL, "nsteps must be positive");
  const int W = h->aw;
  // per stage five events: start, after flags, after limiter, after HWENO, end (2D); the
  // middle three coincide with the start in 1D
  const int ns = 3 * nsteps;
  std::vector<hipEvent_t> ev(5 * ns + 2);
  for (auto& e : ev) HWCHK(hipEventCreate(&e));
  HWCHK(hipEventRecord(ev[5 * ns], h->stream));
  for (int k = 0; k < nsteps; ++k) {
    launch_dt(h, dt > 0.0 ? dt : 0.0, 0.0);
    HWCHK(hipGetLastError());
    const double* ins[3] = {h->S0, h->S1, h->S2};
    double* outs[3] = {h->S1, h->S2, h->S0};
    for (int st = 0; st < 3; ++st) {
      hipEvent_t* e = &ev[5 * (3 * k + st)];
      HWCHK(hipEventRecord(e[0], h->stream));
      if (h->dim == 1)
        for (int m = 1; m <= 3; ++m) HWCHK(hipEventRecord(e[m], h->stream));
      hw_status s = launch_stage(h, hw::MODE_RK1 + st, ins[st], h->S0, outs[st], h->alpha + st * W,
                                 h->alpha + (st + 1) * W, st, nullptr, 0, nullptr,
                                 h->dim == 2 ? e + 1 : nullptr);
      if (s != HW_OK) return s;
      HWCHK(hipEventRecord(e[4], h->stream));
    }
  }
  HWCHK(hipEventRecord(ev[5 * ns + 1], h->stream));
  HWCHK(hipEventSynchronize(ev[5 * ns + 1]));
  double tot = 0.0, part[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < ns; ++k) {
    float ms = 0.f;
    HWCHK(hipEventElapsedTime(&ms, ev[5 * k], ev[5 * k + 4]));
    tot += ms;
    for (int m = 0; m < 4; ++m) {
      HWCHK(hipEventElapsedTime(&ms, ev[5 * k + m], ev[5 * k + m + 1]));
      part[m] += ms;
    }
  }
  float all = 0.f;
  HWCHK(hipEventElapsedTime(&all, ev[5 * ns], ev[5 * ns + 1]));
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (ms_stage) *ms_stage = tot / ns;
  if (ms_step) *ms_step = all / nsteps;
  if (ms_kernels)
    for (int m = 0; m < 4; ++m) ms_kernels[m] = part[m] / ns;
  return HW_OK;
}

// ------------------------------------------------------------------------------ reverse mode
// Checkpoints every k steps; the backward pass walks the segments last to first, replays
// each from its checkpoint with the same stage kernels (so flags, limited moments and
// speeds are reproduced bit for bit), keeping its stage inputs, then runs the stage
// reverses of eq. RK last stage first:
//   stage 3:  G = 2/3 lam + 2/3 dt L2^T lam,   acc  = 1/3 lam,   lam2 = Lim2^T G
//   stage 2:  G = 1/4 lam2 + 1/4 dt L1^T lam2, acc += 3/4 lam2,  lam1 = Lim1^T G
//   stage 1:  G = acc + lam1 + dt L0^T lam1,                     lam  = Lim0^T G
// where acc is the running cotangent of the limited u^n.

static hw_status adjoint_supported(hw_solver* h) {
  if (h->dim != 2 || h->ninst != 1) return fail(h, HW_EINVAL, "reverse mode needs a 2D handle");
  auto wall = [](int bc) {
    return bc == HW_BC_PERIODIC || bc == HW_BC_TRANSMISSIVE || bc == HW_BC_REFLECTIVE;
  };
  if (h->cfg.eq == HW_EULER) {
    const bool step = h->cfg.bc_x == HW_BC_STEP && h->cfg.bc_y == HW_BC_STEP;
    const bool dmrb = h->cfg.bc_x == HW_BC_DMR && h->cfg.bc_y == HW_BC_DMR;
    if (dmrb && h->cfg.tc_mode == HW_TC_NONE)
      return fail(h, HW_EINVAL, "the reverse mode on the double Mach reflection needs troubled-cell detection");
    if (!step && !dmrb && (!wall(h->cfg.bc_x) || !wall(h->cfg.bc_y)))
      return fail(h, HW_EINVAL, "the Euler reverse mode needs periodic, transmissive, reflective, double Mach reflection or forward-step boundaries");
  } else if ((h->cfg.bc_x != HW_BC_PERIODIC && h->cfg.bc_x != HW_BC_TRANSMISSIVE) ||
             (h->cfg.bc_y != HW_BC_PERIODIC && h->cfg.bc_y != HW_BC_TRANSMISSIVE)) {
    return fail(h, HW_EINVAL, "the scalar reverse mode needs periodic or transmissive boundaries");
  }
  return HW_OK;
}

static hw_status ensure_adj_work(hw_solver* h) {
  const size_t st = (size_t)h->nmom * h->nc * h->ncell * sizeof(double);
  double** bufs[4] = {&h->lam, &h->mu, &h->G, &h->acc};
  for (double** b : bufs)
    if (!*b) HWCHK(hipMalloc(b, st));
  if (h->cfg.eq == HW_EULER) {
    const size_t cell = (size_t)h->ncell * sizeof(double);
    if (!h->adjD) HWCHK(hipMalloc(&h->adjD, 4 * 19 * cell));
    if (!h->adjC) HWCHK(hipMalloc(&h->adjC, 2 * 5 * 4 * cell));
    if (!h->adjE) HWCHK(hipMalloc(&h->adjE, 2 * 2 * (size_t)h->cfg.ng_edge * 4 * cell));
  }
  return HW_OK;
}

// rec (Euler with detection, may be null): the stage's recorded list-pass results, read in
// place of rerunning the passes on the stage input
static hw_status launch_adj(hw_solver* h, const double* in, const double* lam, const double* acc_in,
                            double* acc_out, double* out, const unsigned long long* alpha, double cg,
                            double cl, double ca, double kl, int acc_mode,
                            const StageRec* rec = nullptr) {
  hw::Adj2D P{};
  P.in = in; P.lam = lam; P.acc_in = acc_in; P.acc_out = acc_out; P.out = h->G;
  P.alpha = alpha;
  P.cg = cg; P.cl = cl; P.ca = ca; P.kl = kl; P.acc_mode = acc_mode;
  P.nx = h->cfg.nx; P.ny = h->cfg.ny; P.tc_mode = h->cfg.tc_mode;
  P.bcx = h->cfg.bc_x; P.bcy = h->cfg.bc_y;
  step_geometry(&h->cfg, &P.si, &P.sj, P.uin);
  P.x0 = h->cfg.x0;
  P.dtab = (rec && rec->dtab) ? rec->dtab : h->dtab;   // the stage's prescribed ghosts
  P.dx = (h->cfg.x1 - h->cfg.x0) / h->cfg.nx;
  P.dy = (h->cfg.y1 - h->cfg.y0) / h->cfg.ny;
  P.h = 0.5 * std::sqrt(P.dx * P.dx + P.dy * P.dy);
  P.adv0 = h->cfg.adv[0]; P.adv1 = h->cfg.adv[1];
  P.w = h->w;
  if (h->cfg.eq == HW_EULER) {
    // the forward prepasses on the stage input give its flags, limited moments, hybrid
    // masks and HWENO edge values, exactly as the forward pass saw them
    const bool tc = h->cfg.tc_mode != HW_TC_NONE;
    if (tc && rec) {
      P.T = rec->T; P.H = rec->H; P.lim = rec->lim; P.hwv = rec->hwv;
      P.counts = rec->wl; P.flist = rec->wl + 2; P.hlist = rec->wl + 2 + h->ncell;
      P.lens = rec->stats + rec->st;
    } else if (tc) {
      hw::Stage2D F{};
      F.in = in; F.base = in; F.mode = hw::MODE_L;
      F.Tn = h->Tn; F.limn = h->limn;
      F.Tcur = h->Ts; F.Hcur = h->Hs; F.limcur = h->lims; F.G = h->hwv;
      F.counts = h->wl; F.flist = h->wl + 2; F.hlist = h->wl + 2 + h->ncell; F.stats = h->stats;
      F.alpha_in = alpha; F.dt = h->dt; F.status = h->status;
      F.nx = P.nx; F.ny = P.ny; F.bcx = h->cfg.bc_x; F.bcy = h->cfg.bc_y;
      F.tc_mode = h->cfg.tc_mode;
      F.dx = P.dx; F.dy = P.dy; F.h = P.h; F.idx = 1.0 / P.dx; F.idy = 1.0 / P.dy;
      F.gam = h->cfg.gamma_gas; F.x0 = h->cfg.x0; F.y0 = h->cfg.y0; F.t = h->t; F.dtab = h->dtab;
      F.si = P.si; F.sj = P.sj;
      for (int c = 0; c < 4; ++c) F.uin[c] = P.uin[c];
      F.w = h->w;
      HWCHK(hw_launch_prepass2d(h->cfg.eq, h->cfg.ng_edge, &F, h->stream));
      P.T = h->Ts; P.H = h->Hs; P.lim = h->lims; P.hwv = h->hwv;
      P.counts = h->wl; P.flist = h->wl + 2; P.hlist = h->wl + 2 + h->ncell;
    }
    P.gam = h->cfg.gamma_gas;
    P.D = h->adjD; P.E = h->adjE; P.C = h->adjC;
    P.gw = h->G;
    P.out = out;
    HWCHK(hw_launch_adj2d_euler(h->cfg.ng_edge, &P, h->stream));
    return HW_OK;
  }
  HWCHK(hw_launch_adj2d(h->cfg.eq, h->cfg.ng_edge, &P, h->stream));
  P.lam = h->G;
  P.out = out;
  HWCHK(hw_launch_adjlim2d(h->cfg.eq, &P, h->stream));
  return HW_OK;
}

extern "C" hw_status hw_apply_operator_adjoint(hw_solver* h, const double* d_in, const double* d_lambda,
                                               double* d_out) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!d_in || !d_lambda || !d_out) return fail(h, HW_EINVAL, "null device array");
  if (d_out == d_in || d_out == d_lambda) return fail(h, HW_EINVAL, "output must not alias an input");
  hw_status s = adjoint_supported(h);
  if (s != HW_OK || (s = ensure_adj_work(h)) != HW_OK) return s;
  if ((s = launch_alpha(h, d_in, h->alpha_op)) != HW_OK) return s;
  return launch_adj(h, d_in, d_lambda, nullptr, nullptr, d_out, h->alpha_op, 0.0, 1.0, 0.0, 0.0, 0);
}

extern "C" hw_status hw_forward_ckpt(hw_solver* h, int nsteps, double dt, int k) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  hw_status s = adjoint_supported(h);
  if (s != HW_OK) return s;
  if (nsteps <= 0 || k <= 0) return fail(h, HW_EINVAL, "nsteps and k must be positive");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, HW_EINVAL, "dt must be positive and finite");
  h->adj_ready = false;
  const size_t st = (size_t)h->nmom * h->nc * h->ncell;
  const int nck = (nsteps + k - 1) / k;
  if (nck != h->adj_nck) {
    if (h->ckpt) HWCHK(hipFree(h->ckpt));
    h->ckpt = nullptr;
    h->adj_nck = 0;
    HWCHK(hipMalloc(&h->ckpt, nck * st * sizeof(double)));
    h->adj_nck = nck;
  }
  if (k != h->adj_k) {
    if (h->hist) HWCHK(hipFree(h->hist));
    if (h->ahist) HWCHK(hipFree(h->ahist));
    h->hist = nullptr;
    h->ahist = nullptr;
    h->adj_k = 0;
    HWCHK(hipMalloc(&h->hist, (3 * (size_t)k + 1) * st * sizeof(double)));
    HWCHK(hipMalloc(&h->ahist, (3 * (size_t)k + 1) * h->aw * sizeof(unsigned long long)));
    if (h->cfg.eq == HW_EULER && h->cfg.tc_mode != HW_TC_NONE) {
      for (void* p : {(void*)h->recT, (void*)h->recH, (void*)h->recLim, (void*)h->recHwv, (void*)h->recWl,
                      (void*)h->recStats})
        if (p) HWCHK(hipFree(p));
      h->recT = h->recH = nullptr;
      h->recLim = h->recHwv = nullptr;
      h->recWl = nullptr;
      h->recStats = nullptr;
      const size_t ns = 3 * (size_t)k, n = h->ncell;
      HWCHK(hipMalloc(&h->recT, ns * n));
      HWCHK(hipMalloc(&h->recH, ns * n));
      HWCHK(hipMalloc(&h->recLim, ns * (size_t)(h->nmom - 1) * h->nc * n * sizeof(double)));
      HWCHK(hipMalloc(&h->recHwv, ns * 4 * (size_t)h->cfg.ng_edge * h->nc * n * sizeof(double)));
      HWCHK(hipMalloc(&h->recWl, ns * (2 + 2 * n) * sizeof(int)));
      HWCHK(hipMalloc(&h->recStats, (size_t)k * 6 * sizeof(long long)));
      if (h->recDtab) HWCHK(hipFree(h->recDtab));
      h->recDtab = nullptr;
      if (h->cfg.bc_x == HW_BC_DMR)
        HWCHK(hipMalloc(&h->recDtab, ns * 12 * (size_t)hw::dmr::ring2_size(h->cfg.nx, h->cfg.ny) * sizeof(double)));
      // the flags pass appends to each slot's lists; the stage kernel empties them again
      for (size_t r = 0; r < ns; ++r)
        HWCHK(hipMemsetAsync(h->recWl + r * (2 + 2 * n), 0, 2 * sizeof(int), h->stream));
    }
    h->adj_k = k;
  }
  if (!h->adt) HWCHK(hipMalloc(&h->adt, sizeof(double)));
  const bool dmrb = h->cfg.bc_x == HW_BC_DMR;
  if (dmrb && nsteps > h->adj_ntimes) {
    if (h->adj_times) HWCHK(hipFree(h->adj_times));
    h->adj_times = nullptr;
    h->adj_ntimes = 0;
    HWCHK(hipMalloc(&h->adj_times, (size_t)nsteps * sizeof(double)));
    h->adj_ntimes = nsteps;
  }
  if ((s = ensure_adj_work(h)) != HW_OK) return s;
  h->adj_dt = dt;
  HWCHK(hipMemcpyAsync(h->adt, &h->adj_dt, sizeof(double), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipMemsetAsync(h->status, 0, sizeof(int), h->stream));
  for (int n = 0; n < nsteps; ++n) {
    if (n % k == 0)
      HWCHK(hipMemcpyAsync(h->ckpt + (size_t)(n / k) * st, h->S0, st * sizeof(double),
                           hipMemcpyDeviceToDevice, h->stream));
    if ((s = enqueue_step(h, dt, 0.0, 0)) != HW_OK) return s;
    // the step's time after its dt update: the prescribed data of its stages in the replay
    if (dmrb)
      HWCHK(hipMemcpyAsync(h->adj_times + n, h->t, sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  }
  int bad = 0;
  if ((s = read_status(h, &bad)) != HW_OK) return s;
  if (bad) return fail(h, HW_ENONFINITE, "non-finite value in the recorded forward run");
  h->adj_nsteps = nsteps;
  h->adj_ready = true;
  return HW_OK;
}

extern "C" hw_status hw_adjoint(hw_solver* h, const double* d_lambda_T, double* d_grad_U0) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (!d_lambda_T || !d_grad_U0) return fail(h, HW_EINVAL, "null device array");
  if (!h->adj_ready) return fail(h, HW_ESTATE, "no recorded forward run (call hw_forward_ckpt)");
  const size_t st = (size_t)h->nmom * h->nc * h->ncell;
  const int k = h->adj_k;
  const double dt = h->adj_dt;
  HWCHK(hipMemcpyAsync(h->lam, d_lambda_T, st * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  hw_status s;
  for (int seg = h->adj_nck - 1; seg >= 0; --seg) {
    const int n0 = seg * k;
    const int m = std::min(k, h->adj_nsteps - n0);
    // replay the segment, keeping its stage inputs and speeds
    HWCHK(hipMemcpyAsync(h->hist, h->ckpt + (size_t)seg * st, st * sizeof(double),
                         hipMemcpyDeviceToDevice, h->stream));
    const int na = (3 * m + 1) * h->aw;
    hipLaunchKernelGGL(zero_u64, dim3((na + 255) / 256), dim3(256), 0, h->stream, h->ahist, na);
    HWCHK(hipGetLastError());
    if ((s = launch_alpha(h, h->hist, h->ahist)) != HW_OK) return s;
    const bool rec = h->recT != nullptr;
    for (int i = 0; i < m; ++i) {
      double* S = h->hist + 3 * (size_t)i * st;
      const int aw = h->aw;
      unsigned long long* a = h->ahist + 3 * (size_t)i * aw;
      StageRec r0, r1, r2;
      if (rec) {
        r0 = stage_rec(h, 3 * i);
        r1 = stage_rec(h, 3 * i + 1);
        r2 = stage_rec(h, 3 * i + 2);
        if (h->adj_times) r0.t = r1.t = r2.t = h->adj_times + n0 + i;
      }
      if ((s = launch_stage(h, hw::MODE_RK1, S, S, S + st, a, a + aw, -1, nullptr, 0, h->adt, nullptr,
                            rec ? &r0 : nullptr)) != HW_OK) return s;
      if ((s = launch_stage(h, hw::MODE_RK2, S + st, S, S + 2 * st, a + aw, a + 2 * aw, -1, nullptr, 0, h->adt,
                            nullptr, rec ? &r1 : nullptr)) != HW_OK) return s;
      if ((s = launch_stage(h, hw::MODE_RK3, S + 2 * st, S, S + 3 * st, a + 2 * aw, a + 3 * aw, -1, nullptr, 0,
                            h->adt, nullptr, rec ? &r2 : nullptr)) != HW_OK) return s;
    }
    // reverse the segment's steps
    for (int i = m - 1; i >= 0; --i) {
      const double* S = h->hist + 3 * (size_t)i * st;
      const int aw = h->aw;
      const unsigned long long* a = h->ahist + 3 * (size_t)i * aw;
      StageRec r0, r1, r2;
      if (rec) {
        r0 = stage_rec(h, 3 * i);
        r1 = stage_rec(h, 3 * i + 1);
        r2 = stage_rec(h, 3 * i + 2);
      }
      if ((s = launch_adj(h, S + 2 * st, h->lam, nullptr, h->acc, h->mu, a + 2 * aw, 2.0 / 3.0,
                          (2.0 / 3.0) * dt, 0.0, 1.0 / 3.0, 1, rec ? &r2 : nullptr)) != HW_OK) return s;
      if ((s = launch_adj(h, S + st, h->mu, h->acc, h->acc, h->mu, a + aw, 0.25, 0.25 * dt, 0.0,
                          0.75, 2, rec ? &r1 : nullptr)) != HW_OK) return s;
      if ((s = launch_adj(h, S, h->mu, h->acc, nullptr, h->lam, a, 1.0, dt, 1.0, 0.0, 0,
                          rec ? &r0 : nullptr)) != HW_OK) return s;
    }
  }
  HWCHK(hipMemcpyAsync(d_grad_U0, h->lam, st * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return HW_OK;
}

// ------------------------------------------------------------------------------ batched

// one captured graph of nsteps steps (each: dt kernel + three stages)
static hw_status capture_graph(hw_solver* h, double fixed_dt, double T_end, int persistent,
                               int nsteps, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HWCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hw_status s = HW_OK;
  for (int k = 0; k < nsteps && s == HW_OK; ++k) s = enqueue_step(h, fixed_dt, T_end, persistent);
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (s != HW_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  HWCHK(e);
  return HW_OK;
}

// the one-step graph for these parameters, and the multi-step one when nsteps needs it
static hw_status capture_step(hw_solver* h, double fixed_dt, double T_end, int persistent,
                              long nsteps) {
  if (!(h->graph && h->graph_dt == fixed_dt && h->graph_T == T_end && h->graph_persist == persistent &&
        h->graph_grid == h->pgrid && h->graph_tile == h->tile1d)) {
    drop_graph(h);
    hw_status s = capture_graph(h, fixed_dt, T_end, persistent, 1, &h->graph);
    if (s != HW_OK) {
      drop_graph(h);
      return s;
    }
    h->graph_dt = fixed_dt;
    h->graph_T = T_end;
    h->graph_persist = persistent;
    h->graph_grid = h->pgrid;
    h->graph_tile = h->tile1d;
  }
  if (nsteps >= STEPS_PER_GRAPH && !h->graphk) {
    hw_status s = capture_graph(h, fixed_dt, T_end, persistent, STEPS_PER_GRAPH, &h->graphk);
    if (s != HW_OK) {
      drop_graph(h);
      return s;
    }
  }
  return HW_OK;
}

extern "C" hw_status hw_batch_steps(hw_solver* h, int nsteps, int persistent) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (h->dim != 1 || nsteps < 0) return fail(h, HW_EINVAL, "batched steps need a 1D handle and nsteps >= 0");
  const int form = persistent < 0 ? h->auto_persist : (persistent ? 1 : 0);
  hw_status s = capture_step(h, 0.0, 0.0, form, nsteps);
  if (s != HW_OK) return s;
  return launch_steps(h, nsteps);
}

// ------------------------------------------------------------------------------ meshes
extern "C" hw_status hw_set_mesh_1d(hw_solver* h, const double* faces) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (h->dim != 1) return fail(h, HW_EINVAL, "cells of different sizes need a one-dimensional handle");
  const int ni = h->ninst, total = (int)h->ncell;
  // per instance: the smallest cell (the CFL step follows it)
  std::vector<double> dmin(ni);
  if (!faces) {
    // back to the configuration's uniform meshes
    if (h->nu) HWCHK(hipFree(h->nu));
    h->nu = nullptr;
    dmin = h->h_dxs;
  } else {
    for (int b = 0; b < ni; ++b) {
      const double* f = faces + h->h_off[b] + b;
      dmin[b] = HUGE_VAL;
      for (int i = 0; i < h->h_off[b + 1] - h->h_off[b]; ++i) {
        const double d = f[i + 1] - f[i];
        if (!std::isfinite(f[i]) || !std::isfinite(f[i + 1]) || !(d > 0.0))
          return fail(h, HW_EINVAL, "face coordinates must be finite and strictly increasing");
        dmin[b] = std::min(dmin[b], d);
      }
    }
    if (!h->nu) HWCHK(hipMalloc(&h->nu, (size_t)hw::mesh1d::NTAB * total * sizeof(double)));
    double* d_faces = nullptr;
    const size_t nf = (size_t)total + ni;
    HWCHK(hipMalloc(&d_faces, nf * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d_faces, faces, nf * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hw_launch_mesh1d_setup_batch(d_faces, h->h_off.data(), ni, h->cfg.bc_x, h->nu, total, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d_faces);
    HWCHK(e);
    if (h->tile1d != 256 || h->pgrid != 0) {
      hw_status s = build_items(h, 256);
      if (s != HW_OK) return s;
      h->pgrid = 0;
    }
    h->auto_persist = 0;
  }
  // captured steps hold the old kernel arguments
  HWCHK(hipMemcpyAsync(h->dxs, dmin.data(), ni * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  drop_graph(h);
  return HW_OK;
}

extern "C" hw_status hw_batch_set_form(hw_solver* h, int tile, int persistent, int grid) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (h->dim != 1) return fail(h, HW_EINVAL, "launch forms apply to 1D handles");
  if (h->nu) return fail(h, HW_EINVAL, "a mesh of cells of different sizes has one launch form");
  if (tile != 64 && tile != 128 && tile != 256 && tile != 512)
    return fail(h, HW_EINVAL, "tile width must be 64, 128, 256 or 512");
  if (persistent != 0 && persistent != 1) return fail(h, HW_EINVAL, "persistent must be 0 or 1");
  if (persistent && grid < 1) return fail(h, HW_EINVAL, "a persistent grid needs at least one workgroup");
  hw_status s = build_items(h, tile);
  if (s != HW_OK) return s;
  h->pgrid = persistent ? grid : 0;
  h->auto_persist = persistent;
  drop_graph(h);
  return HW_OK;
}

extern "C" hw_status hw_batch_tune(hw_solver* h, int* grid_chosen) {
  if (!h) return fail(nullptr, HW_EINVAL, "null handle");
  if (h->dim != 1) return fail(h, HW_EINVAL, "tuning applies to 1D batches");
  if (h->nu) return fail(h, HW_EINVAL, "a mesh of cells of different sizes has one launch form");
  hipDeviceProp_t prop;
  int dev = 0;
  HWCHK(hipGetDevice(&dev));
  HWCHK(hipGetDeviceProperties(&prop, dev));
  const int cu = prop.multiProcessorCount;
  // snapshot the state: tuning steps must not change it
  const size_t n = (size_t)h->nmom * h->nc * h->ncell;
  const int W = h->aw;
  std::vector<unsigned long long> asave(W);
  HWCHK(hipMemcpyAsync(h->backup, h->S0, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HWCHK(hipMemcpyAsync(asave.data(), h->alpha + 3 * W, W * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  std::vector<double> tsave(h->ninst);
  std::vector<long long> ssave(h->ninst);
  HWCHK(hipMemcpyAsync(tsave.data(), h->t, h->ninst * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipMemcpyAsync(ssave.data(), h->steps, h->ninst * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  // candidates: tile width (= waves per workgroup x 64) x launch form (one workgroup per
  // tile, or a persistent grid of cu x m workgroups walking the work list)
  const int tiles[] = {64, 128, 256, 512};
  const int mults[] = {0, 1, 2, 4, 8};   // 0: one workgroup per tile
  double best = 1e300;
  int best_tile = 256, best_persist = 0, best_grid = 0;
  hipEvent_t e0, e1;
  HWCHK(hipEventCreate(&e0));
  HWCHK(hipEventCreate(&e1));
  hw_status s = HW_OK;
  for (int tile : tiles) {
    if ((s = build_items(h, tile)) != HW_OK) break;
    for (int m : mults) {
      const int persist = m > 0 ? 1 : 0;
      const int grid = persist ? std::min(cu * m, std::max(1, h->nitems)) : 0;
      if (persist && grid >= h->nitems) continue;   // no better than one workgroup per tile
      h->pgrid = grid;
      if ((s = hw_batch_steps(h, 1, persist)) != HW_OK) break;   // capture + warm-up
      HWCHK(hipEventRecord(e0, h->stream));
      if ((s = hw_batch_steps(h, 3, persist)) != HW_OK) break;
      HWCHK(hipEventRecord(e1, h->stream));
      HWCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HWCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_tile = tile;
        best_persist = persist;
        best_grid = grid;
      }
    }
    if (s != HW_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != HW_OK) return s;
  if ((s = build_items(h, best_tile)) != HW_OK) return s;
  h->pgrid = best_grid;
  h->auto_persist = best_persist;
  drop_graph(h);
  HWCHK(hipMemcpyAsync(h->S0, h->backup, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HWCHK(hipMemcpyAsync(h->alpha + 3 * W, asave.data(), W * sizeof(unsigned long long), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipMemcpyAsync(h->t, tsave.data(), h->ninst * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipMemcpyAsync(h->steps, ssave.data(), h->ninst * sizeof(long long), hipMemcpyHostToDevice, h->stream));
  HWCHK(hipStreamSynchronize(h->stream));
  if (grid_chosen) {
    grid_chosen[0] = best_tile;
    grid_chosen[1] = best_persist;
    grid_chosen[2] = best_grid;
  }
  return HW_OK;
}

// ------------------------------------------------------------------ no-allocation operator
// hw_apply_operator_noalloc keeps everything its kernels need beyond the caller's input and
// output (speeds, time-step slot, status, list counters and statistics, flags, hybrid
// masks, work lists, limited moments, HWENO edge values) in one file-scope device array.
// Each GPU holds its own copy from the library's load until the process ends.  In host
// code the array's name is not a device address: the address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that
// address is handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;   // must match include/hweno.h
static_assert(NOALLOC_SCRATCH_BYTES == (size_t)HW_NOALLOC_SCRATCH_BYTES, "scratch size");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr size_t NOALLOC_HEADER = 2048;   // speeds, dt, statistics, status, list counters
std::mutex g_scratch_mutex;
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

__global__ void noalloc_clear(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte offsets of the operator's buffers inside the scratch array for one configuration.
struct NoallocLayout {
  size_t Ts, Hs, flist, hlist, lims, hwv, total;
};

NoallocLayout noalloc_layout(const hw_config* c) {
  const size_t cells = (size_t)c->nx * c->ny;
  const size_t nc = c->eq == HW_EULER ? 4 : 1;
  NoallocLayout L{};
  size_t o = NOALLOC_HEADER;
  if (c->tc_mode != HW_TC_NONE) {
    L.Ts = o; o += align256(cells);
    L.Hs = o; o += align256(cells);
    L.flist = o; o += align256(cells * sizeof(int));
    L.hlist = o; o += align256(cells * sizeof(int));
    L.lims = o; o += align256(2 * nc * cells * sizeof(double));
    L.hwv = o; o += align256((size_t)4 * c->ng_edge * nc * cells * sizeof(double));
  }
  L.total = o;
  return L;
}

// The scratch array's address on the current device (looked up on the first call there).
hipError_t scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" hw_status hw_apply_operator_noalloc(const hw_config* cfg, const double* d_in, double* d_L,
                                               double* d_lim, void* stream) {
  hw_solver* h = nullptr;   // for HWCHK: errors are global
  if (!cfg || !d_in || !d_L) return fail(nullptr, HW_EINVAL, "null argument");
  std::string msg;
  if (validate(cfg, msg) != HW_OK) return fail(nullptr, HW_EINVAL, msg);
  if (cfg->dim != 2) return fail(nullptr, HW_EINVAL, "the no-allocation operator is two-dimensional");
  if (cfg->bc_x == HW_BC_DMR)
    return fail(nullptr, HW_EINVAL, "time-dependent boundary data need a solver handle (hw_apply_operator)");
  if (cfg->bc_x == HW_BC_STEP)
    return fail(nullptr, HW_EINVAL, "the forward-step boundaries need a solver handle (hw_apply_operator)");
  const NoallocLayout lay = noalloc_layout(cfg);
  if (lay.total > NOALLOC_SCRATCH_BYTES)
    return fail(nullptr, HW_EINVAL,
                "mesh needs " + std::to_string(lay.total) + " bytes of scratch; the no-allocation "
                "operator has " + std::to_string(NOALLOC_SCRATCH_BYTES));
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HWCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(nullptr, HW_EINVAL, "device index out of range");
  if (s) {
    int sdev = -1;
    HWCHK(hipStreamGetDevice(s, &sdev));
    if (sdev != dev) return fail(nullptr, HW_EINVAL, "the stream belongs to another device than the current one");
  }
  unsigned char* base = nullptr;
  HWCHK(scratch_address(dev, &base));
  // the header starts every call at zero (a fill kernel, so that the call can be captured)
  hipLaunchKernelGGL(noalloc_clear, dim3(1), dim3(256), 0, s, (unsigned long long*)base,
                     (int)(NOALLOC_HEADER / sizeof(unsigned long long)));
  HWCHK(hipGetLastError());
  unsigned long long* alpha = (unsigned long long*)base;                  // [2][ASPREAD]
  double* dtp = (double*)(base + 1024);
  long long* stats = (long long*)(base + 1088);                          // [6]
  int* status = (int*)(base + 1152);
  int* counts = (int*)(base + 1160);                                     // [2]
  HWCHK(hw_launch_alpha2d(cfg->eq, d_in, cfg->nx, cfg->ny, cfg->gamma_gas, cfg->adv[0], cfg->adv[1],
                          cfg->nx, 0, alpha, s));
  hw::Stage2D P{};
  P.in = d_in; P.base = d_in; P.out = d_L;
  if (cfg->tc_mode != HW_TC_NONE) {
    P.Tcur = base + lay.Ts;
    P.Hcur = base + lay.Hs;
    P.limcur = (double*)(base + lay.lims);
    P.G = (double*)(base + lay.hwv);
    P.counts = counts;
    P.flist = (int*)(base + lay.flist);
    P.hlist = (int*)(base + lay.hlist);
    P.stats = stats;
  }
  P.alpha_in = alpha; P.alpha_out = nullptr; P.dt = dtp;
  P.wout = d_lim; P.status = status;
  P.nx = cfg->nx; P.ny = cfg->ny; P.bcx = cfg->bc_x; P.bcy = cfg->bc_y;
  P.tc_mode = cfg->tc_mode; P.mode = hw::MODE_L;
  P.dx = (cfg->x1 - cfg->x0) / cfg->nx;
  P.dy = (cfg->y1 - cfg->y0) / cfg->ny;
  P.h = 0.5 * std::sqrt(P.dx * P.dx + P.dy * P.dy);
  P.idx = 1.0 / P.dx;
  P.idy = 1.0 / P.dy;
  P.gam = cfg->gamma_gas; P.adv0 = cfg->adv[0]; P.adv1 = cfg->adv[1];
  for (int i = 0; i < 3; ++i) P.w.lim[i] = cfg->lim_w[i];
  for (int i = 0; i < 5; ++i) P.w.rec[i] = cfg->rec_w[i];
  P.w.eps = cfg->eps;
  HWCHK(hw_launch_stage2d(cfg->eq, cfg->ng_edge, &P, s, nullptr));
  return HW_OK;
}

extern "C" const char* hw_last_error(const hw_solver* h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}

extern "C" const char* hw_status_string(int s) {
  switch (s) {
    case HW_OK: return "ok";
    case HW_EINVAL: return "invalid argument";
    case HW_ENOMEM: return "out of device memory";
    case HW_EDEVICE: return "HIP runtime error";
    case HW_ENONFINITE: return "non-finite or non-physical state";
    case HW_ESTATE: return "invalid state for this call";
  }
  return "unknown status";
}

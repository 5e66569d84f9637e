// Parameter blocks shared by the host runtime and the stage kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hw {

enum { EQ_ADV = 0, EQ_BURGERS = 1, EQ_EULER = 2 };
enum { TC_KXRCF = 0, TC_NONE = 1, TC_ALL = 2 };
// BC_DMR: the boundaries of the double Mach reflection problem on all four sides (hw_dmr.h);
// BC_STEP: those of the forward-facing step (hw_step.h)
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_DMR = 3, BC_STEP = 4 };
// kernel instances by boundary kind: rectangular meshes (periodic, transmissive,
// reflective sides), the double Mach reflection, the forward step
enum { BK_RECT = 0, BK_DMR = 1, BK_STEP = 2 };
// stage modes: L only (operator), or the three TVD-RK3 stages of eq. RK
enum { MODE_L = 0, MODE_RK1 = 1, MODE_RK2 = 2, MODE_RK3 = 3 };
// A 2D stage's Lax-Friedrichs speed of each direction is kept as ASPREAD partial maxima
// (workgroup b updates entry b % ASPREAD): one address per direction would serialise the
// atomics of thousands of workgroups.  Slot layout [direction][ASPREAD].
constexpr int ASPREAD = 64;

struct Weights {
  double lim[3];   // limiter linear weights gamma_0..2 (Step 1 / Step 4)
  double rec[5];   // reconstruction linear weights (Step 2.1: 3, Step 5.1: 5)
  double eps;      // epsilon of the nonlinear weights
};

// Two-dimensional stage (see stage2d.hip).
struct Stage2D {
  const double* in;       // stage input, [3][nc][ny][nx]
  const double* base;     // u^n (stages 2, 3)
  double* out;            // stage output (stage 3 may alias base)
  uint8_t* Tn;            // flags of u^n: written in stage 1, read by stages 2, 3
  double* limn;           // limited first moments of u^n, [2][nc][ny][nx], flagged cells only
  uint8_t* Tcur;          // this stage's flags (prepass -> main kernel; Tn in stage 1)
  uint8_t* Hcur;          // this stage's hybrid mask (a flag in the 3 x 3 block; prepass ->
                          // main kernel)
  double* limcur;         // this stage's limited first moments, flagged cells (limn in stage 1)
  double* G;              // HWENO edge values of hybrid cells [2 dir][2 side][NG][nc][ny][nx]
  int* counts;            // work-list lengths: flagged cells, hybrid cells (0 between stages)
  int* flist;             // flagged cells (global index)
  int* hlist;             // hybrid cells (global index)
  long long* stats;       // per stage of the last step: flagged [3], hybrid [3] cell counts
  const unsigned long long* alpha_in;   // Lax-Friedrichs speeds of the stage input [2][ASPREAD]
  unsigned long long* alpha_out;        // max accumulator of the output's speeds [2][ASPREAD]
  const double* dt;       // device time step
  uint8_t* flagsT;        // optional export of this stage's flags T
  uint8_t* flagsH;        // optional export of this stage's hybrid mask H
  double* wout;           // optional export of the limited stage input
  int* status;            // bit 0: non-finite output, bit 1: rho <= 0 or p <= 0
  int nx, ny, bcx, bcy, tc_mode, mode;
  double dx, dy, h, gam, adv0, adv1;
  double idx, idy;        // 1/dx, 1/dy
  double x0, y0;          // mesh origin (prescribed boundary data)
  const double* t;        // time of the step (prescribed boundary data; may be null otherwise)
  double* dtab;           // double Mach reflection: the prescribed ghosts' moments at this
                          // stage's time, [3 nc][ring of two ghost layers] (stage2d.hip);
                          // null otherwise
  int si, sj;             // forward step: solid cells gx >= si, gy < sj (else si = nx, sj = 0)
  double uin[4];          // forward step: conserved inflow state
  Weights w;
};

// One-dimensional stage, single or batched (see stage1d.hip).
struct Stage1D {
  const double* in;        // [2][nc][total]  (averages, first moments; instances concatenated)
  const double* base;      // u^n (stages 2, 3)
  double* out;             // stage output (stage 3 may alias base)
  uint8_t* Tn;             // flags of u^n (stage 1 writes, stages 2/3 read)
  double* limn;            // limited first moments of u^n [nc][total], flagged cells only
  const int2* items;       // work list: (instance, first cell of the tile)
  const int* off;          // instance offsets [ninst + 1]
  const double* dxs;       // cell size per instance
  const unsigned long long* alpha_in;   // per instance
  unsigned long long* alpha_out;        // per instance (max accumulator)
  const double* dt;        // per instance (0: instance finished, skip)
  uint8_t* flagsT;         // optional export
  uint8_t* flagsH;         // optional export
  double* wout;            // optional export of the limited stage input (operator mode)
  int* status;             // bit 0 non-finite, bit 1 rho <= 0 or p <= 0
  const double* nu;        // single instance on cells of different sizes: per-cell tables
                           // [mesh1d::NTAB][total] (hw_mesh1d.h); null on a uniform mesh
  int nitems, total, bc, tc_mode, mode;
  double gam, adv;
  Weights w;
};

// Reverse pass of one two-dimensional stage on periodic meshes (see adjoint2d.hip).  For
// scalar equations the first kernel forms
//   out = cg * lam + cl * (dL/dW)^T lam + ca * acc_in      at W = limited stage input,
// and updates the running cotangent of the limited u^n (acc_mode 1: acc_out = kl * lam,
// 2: acc_out = acc_in + kl * lam); the second applies the transposed limiter Jacobian.
// For Euler the same two results come from four launches through the work arrays below.
struct Adj2D {
  const double* in;        // stage input u^(s), [3][ny][nx]
  const double* lam;       // incoming cotangent, [3][ny][nx]
  const double* acc_in;    // running cotangent (read when ca != 0 or acc_mode == 2)
  double* acc_out;         // may alias acc_in
  double* out;             // outgoing cotangent
  const unsigned long long* alpha;   // the stage's Lax-Friedrichs speeds [2][ASPREAD], held fixed
  double cg, cl, ca, kl;
  int acc_mode, nx, ny, tc_mode;
  int bcx, bcy;            // Euler: periodic, transmissive, reflective, the double Mach
                           // reflection or the forward step (scalar: periodic or transmissive)
  int si, sj;              // forward step: solid cells gx >= si, gy < sj (else si = nx, sj = 0)
  double uin[4];           // forward step: conserved inflow state
  const double* dtab;      // double Mach reflection: the stage's prescribed ghosts (hw_dmr.h)
  double x0;               // double Mach reflection: left side of the mesh
  double dx, dy, h, adv0, adv1;
  Weights w;
  // Euler (adjE* kernels): the forward prepasses' results on the stage input, rerun
  // before the reverse, and the work arrays of the reverse
  double gam;
  const uint8_t* T;        // flags of the stage input (null without detection)
  const uint8_t* H;        // hybrid masks (null without detection)
  const double* lim;       // limited first moments of flagged cells [2][4][ny][nx]
  const double* hwv;       // HWENO edge values of hybrid cells [2 dir][2 side][NG][4][ny][nx]
  int* counts;             // forward work-list lengths (flagged, hybrid); zeroed by the reverse
  const long long* lens;   // when not null, the list lengths of a recorded stage instead
                           // (flagged at [0], hybrid at [3]: a stage's entries of stats)
  const int* flist;        // flagged cells
  const int* hlist;        // hybrid cells
  double* D;               // stencil cotangents of every cell [4][19][ny][nx]
  double* E;               // edge-value cotangents of hybrid cells [2 dir][2 NG][4][ny][nx]
  double* C;               // limiter cotangents of flagged cells [2 dir][5][4][ny][nx]
  double* gw;              // cotangent of the limited stage input [3][4][ny][nx]
};

}  // namespace hw

extern "C" {
// ev (may be null): three events recorded after the flags, limiter and HWENO launches
// (for timing each launch; immediately one after another without troubled-cell detection)
hipError_t hw_launch_stage2d(int eq, int ng, const hw::Stage2D* P, hipStream_t s, hipEvent_t* ev);
// cells gx >= si, gy < sj are skipped (solid cells of the forward step; si = nx: none)
hipError_t hw_launch_alpha2d(int eq, const double* U, int nx, int ny, double gam, double a0,
                             double a1, int si, int sj, unsigned long long* alpha_out,
                             hipStream_t s);
// per-cell tables of a single 1D instance on cells of different sizes (hw_mesh1d.h)
hipError_t hw_launch_mesh1d_setup(const double* faces, int n, int bc, double* tab, hipStream_t s);
hipError_t hw_launch_stage1d(int eq, int persistent, int grid, int tile, const hw::Stage1D* P,
                             hipStream_t s);
hipError_t hw_launch_alpha1d(int eq, const double* U, const int* off, int ninst, int total,
                             int maxn, double gam, double adv, unsigned long long* alpha_out,
                             hipStream_t s);
hipError_t hw_launch_adj2d(int eq, int ng, const hw::Adj2D* P, hipStream_t s);
hipError_t hw_launch_adjlim2d(int eq, const hw::Adj2D* P, hipStream_t s);
// 2D Euler: the four reverse launches of one stage (after the forward prepasses)
hipError_t hw_launch_adj2d_euler(int ng, const hw::Adj2D* P, hipStream_t s);
// the forward prepasses of a 2D stage only (flags and work lists, limiter, HWENO values)
hipError_t hw_launch_prepass2d(int eq, int ng, const hw::Stage2D* P, hipStream_t s);
}

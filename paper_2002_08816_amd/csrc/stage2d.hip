// Two-dimensional stage of the hybrid Hermite WENO scheme (Zhao & Qiu, arXiv 2002.08816,
// Section 2.2, Steps 4-6 and eq. ode2).  Per Runge-Kutta stage, with troubled-cell
// detection on, four launches:
//
//  stage2d_flags  per 16 x 16 tile: KXRCF flags (Step 4, Remark 3) of tile+1 from the
//                 fields the indicator reads; writes the tile's flags and hybrid masks
//                 (a flag in the 3 x 3 block, Step 5) and appends its flagged cells and
//                 its hybrid cells to two work lists.
//  stage2d_limit  the Jacobi limiter of the first moments (Step 4, Remark 4) over the
//                 flagged-cell list, one (cell, direction, characteristic field) per thread.
//  stage2d_hweno  the HWENO edge values (Step 5.1) over the hybrid-cell list, one
//                 (cell, characteristic field) per thread, both directions.  Work lists rather than tiles: the few tiles a shock crosses
//                 would otherwise each run their whole share on one compute unit.
//  stage2d_kernel per 16 x 16 tile with two ghost layers (flags, hybrid masks and
//                 limited moments read back): interior Gauss values of the least-squares quartic -> volume
//                 integrals (Step 5.3); per direction, the edge values of the cell and of
//                 its two neighbours (Step 5.2 linear, or the stored HWENO values), the
//                 Lax-Friedrichs fluxes of its two faces and the edge quadratures of eq.
//                 ode2; the TVD-RK3 stage combination (eq. RK) with the limited moments,
//                 the store, and the block's share of the next stage's speeds.  Each cell
//                 evaluates its own edge values once; a neighbour's come from a lane
//                 shuffle, from the LDS row between two waves, or, across the tile's
//                 sides, from the ring cells the tile evaluates once in LDS.  Each face's
//                 flux is then formed by both of its cells from the same values.
// Without detection only stage2d_kernel runs.
//
// The limited first moments of the stage input replace the stored ones in the stage
// combination; the flags and limited moments of u^n (stage 1) are kept for stages 2, 3.
// Ghost cells at transmissive and reflective boundaries are mirror images of the cells
// they copy in every respect (state, flag, hybrid mask, limited moments, edge values); a
// reflective wall also reverses the normal momentum.
#include "hw_dmr.h"
#include "hw_step.h"
#include "hw_tile2d.h"

namespace hw {

// ------------------------------------------------------------------ prepasses
constexpr int H2 = 2, L2 = TX + 2 * H2, NP2 = L2 * L2;   // tile + two ghost layers

// global index of the cell a distance-1 transmissive or reflective ghost mirrors (other
// indices as given)
__device__ __forceinline__ int mirror1(int g, int n, int bc) {
  if (bc == BC_PERIODIC) return g;
  if (g == -1) return 0;
  if (g == n) return n - 1;
  return g;
}

// Factor a reflective wall adds to every value of component c of a ghost cell, on top of
// the mirror's moment signs: the normal momentum (rho u across an x wall, rho v across a y
// wall) is reversed.  xm / ym: the cell is a mirror image across an x / y boundary.
template <int EQ>
__device__ __forceinline__ double wall_factor(int c, bool xm, bool ym, int bcx, int bcy) {
  if constexpr (EQ != EQ_EULER) return 1.0;
  double f = 1.0;
  if (c == 1 && xm && bcx == BC_REFLECTIVE) f = -f;
  if (c == 2 && ym && (bcy == BC_REFLECTIVE || bcy == BC_DMR)) f = -f;
  return f;
}

// double Mach reflection: whether the stencil position (gx, gy) is a prescribed ghost cell,
// and the value of its field f at the stage's time ts.  BK: the boundary kind the kernel
// instance is for (BK_RECT, BK_DMR, BK_STEP); only the instances of the double Mach
// reflection and the forward step carry their boundaries' code.
template <int BK>
__device__ __forceinline__ bool dmr_prescribed(const Stage2D& P, int gx, int gy) {
  if constexpr (BK == BK_DMR) return dmr::prescribed(gx, gy, P.nx, P.ny, P.x0, P.dx);
  return false;
}
// The prescribed ghosts' moments are computed once per stage (dmr_table_kernel) into a
// table over the ring of two ghost layers around the mesh (dmr::ring2_index).
// value of field f of the prescribed ghost (gx, gy) at the stage's time
__device__ __forceinline__ double dmr_value(const Stage2D& P, int f, int gx, int gy, double) {
  return P.dtab[(size_t)f * dmr::ring2_size(P.nx, P.ny) + dmr::ring2_index(gx, gy, P.nx, P.ny)];
}
template <int BK>
__device__ __forceinline__ double stage_time_of(const Stage2D& P, double dtv) {
  if constexpr (BK == BK_DMR) return dmr::stage_time(P.t, dtv, P.mode);
  return 0.0;
}

// Appends the threads marked in a to list a and those marked in b to list b, with one
// atomic per list and workgroup (workgroups with nothing to append touch no counter).
__device__ __forceinline__ void block_append2(bool ma, bool mb, int value, int* counts,
                                              int* list_a, int* list_b,
                                              int* s_wave /* 10 ints */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long a = __ballot(ma), b = __ballot(mb);
  if (lane == 0) {
    s_wave[w] = __popcll(a);
    s_wave[4 + w] = __popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int* sw = s_wave + 4 * threadIdx.x;
    const int tot = sw[0] + sw[1] + sw[2] + sw[3];
    s_wave[8 + threadIdx.x] = tot ? atomicAdd(&counts[threadIdx.x], tot) : 0;
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  if (ma) {
    int off = s_wave[8];
    for (int i = 0; i < w; ++i) off += s_wave[i];
    list_a[off + __popcll(a & below)] = value;
  }
  if (mb) {
    int off = s_wave[9];
    for (int i = 0; i < w; ++i) off += s_wave[4 + i];
    list_b[off + __popcll(b & below)] = value;
  }
}

// KXRCF flags of every cell (Step 4, Remark 3; Euler: density or energy fires).  Each
// tile stages only what the indicator reads, with two ghost layers, and evaluates the
// flags of tile+1 so that it also knows its hybrid cells (a flag in the 3 x 3 block,
// Step 5); transmissive ghosts take the flag of the cell they mirror.  The tile's flags
// and hybrid masks are stored, and its flagged and hybrid cells appended to two work
// lists.
template <int EQ, int BK>
__global__ __launch_bounds__(NT) void stage2d_flags_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int NK = (EQ == EQ_EULER) ? 2 : 1;   // components checked: density, energy
  constexpr int NV = (EQ == EQ_EULER) ? 2 : 0;   // momentum averages (velocity)
  constexpr int NFK = 3 * NK;                    // averages and moments of those
  constexpr int W1 = L2 - 2;                     // tile+1
  __shared__ double s_k[NFK * NP2];
  __shared__ uint8_t s_vs[NP2];                  // Euler: inflow sides (velocity signs)
  __shared__ uint8_t s_T[NP2];
  __shared__ int s_wave[10];

  // zero once the run has reached its final time (nothing to do); checked after the loads
  // of the tile are issued (the pointer is valid in every mode)
  const double dtv = *P.dt;
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - H2, gy0 = by * TY - H2;
  const size_t plane = (size_t)nx * ny;
  // staging: each thread's (at most NR) positions, every load issued before the stores
  constexpr int NR = (NP2 + NT - 1) / NT;
  double kv[NR][NFK + NV];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = tid + r * NT;
    if (q < NP2) {
      const int ly = q / L2, lx = q - ly * L2;
      double sx, sy;
      size_t gs;
      if constexpr (BK == BK_STEP) {
        // forward step: the position's source cell, or the inflow state
        const step::Src sr = step::resolve(gx0 + lx, gy0 + ly, nx, ny, P.si, P.sj);
        if (sr.pres) {
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            kv[r][3 * k] = P.uin[k == 0 ? 0 : NC - 1];
            kv[r][3 * k + 1] = kv[r][3 * k + 2] = 0.0;
          }
#pragma unroll
          for (int k = 0; k < NV; ++k) kv[r][NFK + k] = P.uin[1 + k];
          continue;
        }
        sx = sr.sx;
        sy = sr.sy;
        gs = (size_t)sr.y * nx + sr.x;
      } else {
        const int gx = map_index(gx0 + lx, nx, P.bcx, sx);
        const int gy = map_index(gy0 + ly, ny, P.bcy, sy);
        gs = (size_t)gy * nx + gx;
      }
      if (dmr_prescribed<BK>(P, gx0 + lx, gy0 + ly)) {
        const double ts = stage_time_of<BK>(P, dtv);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          const int c = k == 0 ? 0 : NC - 1;
#pragma unroll
          for (int m = 0; m < 3; ++m) kv[r][3 * k + m] = dmr_value(P, m * NC + c, gx0 + lx, gy0 + ly, ts);
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) kv[r][NFK + k] = dmr_value(P, 1 + k, gx0 + lx, gy0 + ly, ts);
        continue;
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int c = k == 0 ? 0 : NC - 1;
        kv[r][3 * k] = P.in[c * plane + gs];
        kv[r][3 * k + 1] = sx * P.in[(NC + c) * plane + gs];
        kv[r][3 * k + 2] = sy * P.in[(2 * NC + c) * plane + gs];
      }
#pragma unroll
      for (int k = 0; k < NV; ++k) kv[r][NFK + k] = P.in[(1 + k) * plane + gs];
    }
  }
  if (P.mode != MODE_L && dtv == 0.0) return;   // uniform over the grid
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = tid + r * NT;
    if (q < NP2) {
#pragma unroll
      for (int f = 0; f < NFK; ++f) s_k[f * NP2 + q] = kv[r][f];
      if constexpr (EQ == EQ_EULER) {
        // velocity (rho u)/rho, (rho v)/rho at the average: which faces are inflow
        const double velx = kv[r][NFK] / kv[r][0], vely = kv[r][NFK + 1] / kv[r][0];
        s_vs[q] = (uint8_t)((velx > 0.0) | ((velx < 0.0) << 1) | ((vely > 0.0) << 2) |
                            ((vely < 0.0) << 3));
      }
    }
  }
  __syncthreads();
  auto K = [&](int f, int y, int x) { return s_k[f * NP2 + y * L2 + x]; };
  for (int q = tid; q < W1 * W1; q += NT) {
    const int ly = 1 + q / W1, lx = 1 + q % W1;
    uint8_t t = 0;
    if (P.tc_mode == TC_ALL) {
      t = 1;
    } else {
      bool lin, rin, bin, tin;
      if constexpr (EQ == EQ_EULER) {
        const unsigned vs = s_vs[ly * L2 + lx];
        lin = vs & 1u; rin = vs & 2u; bin = vs & 4u; tin = vs & 8u;
      } else {
        const double velx = EQ == EQ_BURGERS ? K(0, ly, lx) : P.adv0;
        const double vely = EQ == EQ_BURGERS ? K(0, ly, lx) : P.adv1;
        lin = velx > 0.0; rin = velx < 0.0; bin = vely > 0.0; tin = vely < 0.0;
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        double cc[3], l[3], r[3], b[3], tt[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          cc[m] = K(3 * k + m, ly, lx);
          l[m] = K(3 * k + m, ly, lx - 1);
          r[m] = K(3 * k + m, ly, lx + 1);
          b[m] = K(3 * k + m, ly - 1, lx);
          tt[m] = K(3 * k + m, ly + 1, lx);
        }
        if (kxrcf2d_in(cc, l, r, b, tt, lin, rin, bin, tin, P.dx, P.dy, P.h)) t = 1;
      }
    }
    s_T[ly * L2 + lx] = t;
  }
  __syncthreads();
  if (P.bcx != BC_PERIODIC || P.bcy != BC_PERIODIC) {
    // ghosts take the flag of the cell they mirror; prescribed ghosts are never troubled
    uint8_t tg[(W1 * W1 + NT - 1) / NT];
#pragma unroll
    for (int r = 0; r < (W1 * W1 + NT - 1) / NT; ++r) {
      const int q = tid + r * NT;
      if (q >= W1 * W1) break;
      const int ly = 1 + q / W1, lx = 1 + q % W1;
      if constexpr (BK == BK_STEP) {
        // the flag of the source cell; a source outside the staged block only belongs to
        // a position that no tile cell's 3 x 3 block holds
        const step::Src sr = step::resolve(gx0 + lx, gy0 + ly, nx, ny, P.si, P.sj);
        const int mx = sr.x - gx0, my = sr.y - gy0;
        tg[r] = (!sr.pres && mx >= 0 && mx < L2 && my >= 0 && my < L2) ? s_T[my * L2 + mx] : 0;
      } else {
        const int mx = mirror1(gx0 + lx, nx, P.bcx) - gx0, my = mirror1(gy0 + ly, ny, P.bcy) - gy0;
        tg[r] = dmr_prescribed<BK>(P, gx0 + lx, gy0 + ly) ? 0 : s_T[my * L2 + mx];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (W1 * W1 + NT - 1) / NT; ++r) {
      const int q = tid + r * NT;
      if (q >= W1 * W1) break;
      const int ly = 1 + q / W1, lx = 1 + q % W1;
      s_T[ly * L2 + lx] = tg[r];
    }
    __syncthreads();
  }
  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + H2, ly = ty + H2;
  const int gx = gx0 + lx, gy = gy0 + ly;
  const bool inmesh = gx < nx && gy < ny;
  // solid cells of the forward step are never flagged
  bool active = inmesh;
  if constexpr (BK == BK_STEP) active = inmesh && !step::solid(gx, gy, P.si, P.sj);
  const int gi = inmesh ? gy * nx + gx : 0;
  uint8_t t = s_T[ly * L2 + lx];
  uint8_t hm = 0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) hm |= s_T[(ly + dy) * L2 + lx + dx];
  if (!active) t = hm = 0;
  if (inmesh) {
    P.Tcur[gi] = t;
    P.Hcur[gi] = hm;
  }
  block_append2(active && t, active && hm, gi, P.counts, P.flist, P.hlist, s_wave);
}

// Value of field f at the cell (gy, gx) + (dy, dx) as the stencil of that cell sees it:
// boundary mapping (transmissive ghosts negate their normal moment), and the limited
// first moment where the cell is flagged.
template <int BK>
__device__ __forceinline__ double stencil_value(const Stage2D& P, int f, int NC, int gy, int gx,
                                                int dy, int dx, bool limited, double ts) {
  if (dmr_prescribed<BK>(P, gx + dx, gy + dy)) return dmr_value(P, f, gx + dx, gy + dy, ts);
  if constexpr (BK == BK_STEP) {
    const step::Src sr = step::resolve(gx + dx, gy + dy, P.nx, P.ny, P.si, P.sj);
    const int m = f / NC, c = f % NC;
    if (sr.pres) return m == 0 ? P.uin[c] : 0.0;
    const size_t plane = (size_t)P.nx * P.ny, g = (size_t)sr.y * P.nx + sr.x;
    const double wf = step::comp_factor(sr, c);
    if (m == 0) return wf * P.in[f * plane + g];
    const double v = (limited && P.Tcur[g]) ? P.limcur[(f - NC) * plane + g] : P.in[f * plane + g];
    return wf * (m == 1 ? sr.sx * v : sr.sy * v);
  }
  double sx, sy;
  const int x = map_index(gx + dx, P.nx, P.bcx, sx);
  const int y = map_index(gy + dy, P.ny, P.bcy, sy);
  const size_t plane = (size_t)P.nx * P.ny, g = (size_t)y * P.nx + x;
  const int m = f / NC;
  const double wf = NC == 4 ? wall_factor<EQ_EULER>(f % NC, sx < 0.0, sy < 0.0, P.bcx, P.bcy) : 1.0;
  if (m == 0) return wf * P.in[f * plane + g];
  const double v = (limited && P.Tcur[g]) ? P.limcur[(f - NC) * plane + g] : P.in[f * plane + g];
  return wf * (m == 1 ? sx * v : sy * v);
}

// Jacobi limiter of the first moments of every flagged cell (Step 4, Remark 4): one work
// item per (cell, direction, characteristic field).  For Euler the four items of one
// (cell, direction) sit on four consecutive lanes; lane f reads component f of the
// stencil, the group exchanges the components to project onto its characteristic
// fields, and exchanges the limited fields to return to component f.
template <int EQ, int BK>
__global__ __launch_bounds__(NT) void stage2d_limit_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  const long long n = (long long)P.counts[0] * 2 * NC;   // whole groups of NC items
  const double dtv = *P.dt;   // loaded together with the list length
  if ((P.mode != MODE_L && dtv == 0.0) || n == 0) return;
  const int lane = threadIdx.x & 63;
  const size_t plane = (size_t)P.nx * P.ny;
  for (long long base = (long long)blockIdx.x * NT + threadIdx.x - lane; base < n;
       base += (long long)gridDim.x * NT) {
    const long long it = base + lane;
    if (it >= n) continue;
    const int f = (int)(it % NC), dir = (int)((it / NC) & 1);
    const int gi = P.flist[(it / NC) >> 1];
    const int gy = gi / P.nx, gx = gi - gy * P.nx;
    const int oy = dir, ox = 1 - dir, mf = 1 + dir;
    // component f of the stencil along dir (unlimited values)
    const double ts = stage_time_of<BK>(P, dtv);
    const double um = stencil_value<BK>(P, f, NC, gy, gx, -oy, -ox, false, ts);
    const double u0 = P.in[f * plane + gi];
    const double up = stencil_value<BK>(P, f, NC, gy, gx, oy, ox, false, ts);
    const double vm = stencil_value<BK>(P, mf * NC + f, NC, gy, gx, -oy, -ox, false, ts);
    const double vp = stencil_value<BK>(P, mf * NC + f, NC, gy, gx, oy, ox, false, ts);
    if constexpr (EQ == EQ_EULER) {
      double U[4], Lr[4], Rr[4], x[4];
      quad_gather(u0, U);
      euler_rows2d(U, P.gam, dir, f, Lr, Rr);
      double cm = 0.0, c0 = 0.0, cp = 0.0, wm = 0.0, wp = 0.0;
      quad_gather(um, x);
#pragma unroll
      for (int c = 0; c < 4; ++c) cm = fma(Lr[c], x[c], cm);
#pragma unroll
      for (int c = 0; c < 4; ++c) c0 = fma(Lr[c], U[c], c0);
      quad_gather(up, x);
#pragma unroll
      for (int c = 0; c < 4; ++c) cp = fma(Lr[c], x[c], cp);
      quad_gather(vm, x);
#pragma unroll
      for (int c = 0; c < 4; ++c) wm = fma(Lr[c], x[c], wm);
      quad_gather(vp, x);
#pragma unroll
      for (int c = 0; c < 4; ++c) wp = fma(Lr[c], x[c], wp);
      const double vc = limit_moment(cm, c0, cp, wm, wp, P.w.lim, P.w.eps);
      quad_gather(vc, x);
      double out = 0.0;
#pragma unroll
      for (int g = 0; g < 4; ++g) out = fma(Rr[g], x[g], out);
      P.limcur[(size_t)(dir * 4 + f) * plane + gi] = out;
    } else {
      P.limcur[(size_t)dir * plane + gi] = limit_moment(um, u0, up, vm, vp, P.w.lim, P.w.eps);
    }
  }
}

// HWENO edge values (Step 5.1) of every hybrid cell, one work item per (cell,
// characteristic field), grouped as in the limiter: lane f reads component f of the
// 19-value stencil (through the cache, with the limited moments of flagged cells), and
// for each direction in turn the group projects onto that direction's characteristic
// fields, reconstructs field f, and returns to component f, which the lane stores.  Each
// wave takes 64 / NC cells; the stencil is loaded once for both directions (the loads,
// scattered over the hybrid cells, are what this pass waits on).
template <int EQ, int NGE, int BK>
__global__ __launch_bounds__(NT, BK == BK_DMR ? 2 : 1) void stage2d_hweno_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int CPW = 64 / NC;   // cells per wave
  // the list length and the time step are loaded together (the time step pointer is valid
  // in every mode); a finished run or an empty list has nothing to do
  const int ncell = P.counts[1];
  const double dtv = *P.dt;
  if ((P.mode != MODE_L && dtv == 0.0) || ncell == 0) return;
  const long long nwave = (ncell + CPW - 1) / CPW;
  const int lane = threadIdx.x & 63;
  const size_t plane = (size_t)P.nx * P.ny;
  // the cross of the first-moment stencil inside the 3 x 3 block
  const int cross[5] = {1, 3, 4, 5, 7};
  for (long long wq = ((long long)blockIdx.x * NT + threadIdx.x) >> 6; wq < nwave;
       wq += ((long long)gridDim.x * NT) >> 6) {
    const long long cell = wq * CPW + lane / NC;
    if (cell >= ncell) continue;   // whole groups of NC lanes
    const int f = lane % NC;
    const int gi = P.hlist[cell];
    const int gy = gi / P.nx, gx = gi - gy * P.nx;
    // the 3 x 3 block: stored index, moment signs (transmissive ghosts)
    int gb[9];
    unsigned neg_x = 0, neg_y = 0, neg_w = 0, pres = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if constexpr (BK == BK_STEP) {
        // forward step: the position's source cell (prescribed: the inflow state, below)
        const step::Src sr = step::resolve(gx + k % 3 - 1, gy + k / 3 - 1, P.nx, P.ny, P.si, P.sj);
        gb[k] = sr.y * P.nx + sr.x;
        if (sr.pres) pres |= 1u << k;
        if (sr.sx < 0.0) neg_x |= 1u << k;
        if (sr.sy < 0.0) neg_y |= 1u << k;
        if (step::comp_factor(sr, f) < 0.0) neg_w |= 1u << k;
      } else {
        double sx, sy;
        const int x = map_index(gx + k % 3 - 1, P.nx, P.bcx, sx);
        const int y = map_index(gy + k / 3 - 1, P.ny, P.bcy, sy);
        gb[k] = y * P.nx + x;
        if (sx < 0.0) neg_x |= 1u << k;
        if (sy < 0.0) neg_y |= 1u << k;
        if (wall_factor<EQ>(f, sx < 0.0, sy < 0.0, P.bcx, P.bcy) < 0.0) neg_w |= 1u << k;
      }
    }
    // component f of the stencil: 9 averages, then x and y moments of the cross; the
    // stored values and the cross cells' flags are loaded together, the limited moments
    // of the (few) flagged cells afterwards
    double in[19];
    uint8_t tf[5];
#pragma unroll
    for (int k = 0; k < 9; ++k) in[k] = P.in[f * plane + gb[k]];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int k = cross[j];
      tf[j] = P.Tcur[gb[k]];
      in[9 + j] = P.in[(NC + f) * plane + gb[k]];
      in[14 + j] = P.in[(2 * NC + f) * plane + gb[k]];
    }
    // forward step: prescribed inflow positions hold the inflow state, zero moments, and
    // are never troubled
    if constexpr (BK == BK_STEP) {
      if (pres) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
          if ((pres >> k) & 1u) in[k] = P.uin[f];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          if (!((pres >> cross[j]) & 1u)) continue;
          tf[j] = 0;
          in[9 + j] = in[14 + j] = 0.0;
        }
      }
    }
    // double Mach reflection: prescribed ghosts of the block hold the exact solution (signs
    // below apply to mirrored ghosts only) and are never troubled
    if constexpr (BK == BK_DMR) {
      const double ts = stage_time_of<BK>(P, dtv);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int bx = gx + k % 3 - 1, by = gy + k / 3 - 1;
        if (!dmr_prescribed<BK>(P, bx, by)) continue;
        pres |= 1u << k;
        in[k] = dmr_value(P, f, bx, by, ts);
      }
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const int k = cross[j];
        if (!((pres >> k) & 1u)) continue;
        tf[j] = 0;
        in[9 + j] = dmr_value(P, NC + f, gx + k % 3 - 1, gy + k / 3 - 1, ts);
        in[14 + j] = dmr_value(P, 2 * NC + f, gx + k % 3 - 1, gy + k / 3 - 1, ts);
      }
      neg_x &= ~pres;
      neg_y &= ~pres;
      neg_w &= ~pres;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int k = cross[j];
      if (tf[j]) {
        in[9 + j] = P.limcur[f * plane + gb[k]];
        in[14 + j] = P.limcur[(NC + f) * plane + gb[k]];
      }
      if ((neg_x ^ neg_w) >> k & 1u) in[9 + j] = -in[9 + j];
      if ((neg_y ^ neg_w) >> k & 1u) in[14 + j] = -in[14 + j];
    }
    // a reflective wall also reverses the normal momentum of its ghost cells
    if (neg_w) {
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if ((neg_w >> k) & 1u) in[k] = -in[k];
    }
    // both directions from the one stencil (the loop is unrolled: the direction is a
    // constant in each copy)
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
    double v[2 * NGE];
    if constexpr (EQ == EQ_EULER) {
      double U[4], Lr[4], Rr[4], x[4];
      quad_gather(in[4], U);   // the cell's own averages
      euler_rows2d(U, P.gam, dir, f, Lr, Rr);
      double w19[19];
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        quad_gather(in[k], x);
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) a = fma(Lr[c], x[c], a);
        w19[k] = a;
      }
      double wv[2 * NGE];
      if (dir == 0) hweno2d_field<NGE>(w19, P.w, 0, wv);   // the direction as a constant
      else hweno2d_field<NGE>(w19, P.w, 1, wv);
#pragma unroll
      for (int k = 0; k < 2 * NGE; ++k) {
        quad_gather(wv[k], x);
        double a = 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) a = fma(Rr[g], x[g], a);
        v[k] = a;
      }
    } else {
      if (dir == 0) hweno2d_field<NGE>(in, P.w, 0, v);
      else hweno2d_field<NGE>(in, P.w, 1, v);
    }
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      P.G[((((size_t)(dir * 2 + 0) * NGE + k) * NC + f)) * plane + gi] = v[k];
      P.G[((((size_t)(dir * 2 + 1) * NGE + k) * NC + f)) * plane + gi] = v[NGE + k];
    }
    __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ------------------------------------------------------------------ main stage kernel

// Edge values of the cell at LDS position (ly, lx) on the faces of direction dir (lo:
// left or bottom, hi: right or top; either may be null): p0 at the edge Gauss points
// (Step 5.2), or for a hybrid cell the values the prepass stored (Step 5.1).  A ghost's
// stored values are those of the cell it mirrors, faces and edge points reflected.
// The 19 stencil values of component c around (ly, lx) as seen along direction dir: for
// dir = 1 the stencil is transposed (x and y offsets swapped, x and y moments swapped),
// so that the y-face values are the x-face map of the transposed stencil.  Every y-face
// value in this kernel is formed this way, so the two cells of a face agree to the bit.
// (DIR = 0 or 1: a direction known at compile time, so that the offsets are immediates;
// DIR = -1: the direction dir of each lane)
template <int NC, int DIR>
__device__ __forceinline__ void gather19_dir(const double* s, int c, int ly, int lx, int dir,
                                             double* in) {
  if constexpr (DIR >= 0) dir = DIR;
  const int sa = dir == 0 ? L2 : 1, sb = dir == 0 ? 1 : L2;   // strides of dy, dx
  const double* p = s + c * NP2 + ly * L2 + lx;
#pragma unroll
  for (int k = 0; k < 9; ++k) in[k] = p[(k / 3 - 1) * sa + (k % 3 - 1) * sb];
  const double* pv = p + (dir == 0 ? NC : 2 * NC) * NP2;   // moment along dir
  const double* pw = p + (dir == 0 ? 2 * NC : NC) * NP2;   // the other moment
  const int cy[5] = {-1, 0, 0, 0, 1}, cx[5] = {0, -1, 0, 1, 0};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    in[9 + j] = pv[cy[j] * sa + cx[j] * sb];
    in[14 + j] = pw[cy[j] * sa + cx[j] * sb];
  }
}

template <int NGE>
__device__ __forceinline__ void lin_xfaces(const double* in, double* lo, double* hi) {
  if constexpr (NGE == 2) hw2::lin2d_xedges_ng2(in, lo, hi);
  else hw2::lin2d_xedges_ng3(in, lo, hi);
}

template <int EQ, int NGE, int DIR, int BK>
__device__ __forceinline__ void cell_traces(const Stage2D& P, const double* s_u, bool hyb, int ly,
                                            int lx, int dir, int gx0, int gy0, double (*lo)[NGE],
                                            double (*hi)[NGE]) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  if constexpr (DIR >= 0) dir = DIR;
  if (!hyb) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19], a[NGE], b[NGE];
      gather19_dir<NC, DIR>(s_u, c, ly, lx, dir, in);
      lin_xfaces<NGE>(in, a, b);
#pragma unroll
      for (int k = 0; k < NGE; ++k) {
        if (lo) lo[c][k] = a[k];
        if (hi) hi[c][k] = b[k];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  double sx, sy, fu = 1.0, fv = 1.0;
  int gx, gy;
  if constexpr (BK == BK_STEP) {
    const step::Src sr = step::resolve(gx0 + lx, gy0 + ly, P.nx, P.ny, P.si, P.sj);
    gx = sr.x;
    gy = sr.y;
    sx = sr.sx;
    sy = sr.sy;
    fu = sr.fu;
    fv = sr.fv;
  } else {
    gx = map_index(gx0 + lx, P.nx, P.bcx, sx);
    gy = map_index(gy0 + ly, P.ny, P.bcy, sy);
  }
  const bool mx = sx < 0.0, my = sy < 0.0;
  const bool swap = dir == 0 ? mx : my, flip = dir == 0 ? my : mx;
  const size_t plane = (size_t)P.nx * P.ny, gi = (size_t)gy * P.nx + gx;
  const int slo = swap ? 1 : 0, shi = 1 - slo;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double wf;
    if constexpr (BK == BK_STEP) wf = c == 1 ? fu : (c == 2 ? fv : 1.0);
    else wf = wall_factor<EQ>(c, mx, my, P.bcx, P.bcy);
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      const int kk = flip ? NGE - 1 - k : k;
      if (lo) lo[c][k] = wf * P.G[((((size_t)(dir * 2 + slo) * NGE + kk) * NC + c)) * plane + gi];
      if (hi) hi[c][k] = wf * P.G[((((size_t)(dir * 2 + shi) * NGE + kk) * NC + c)) * plane + gi];
    }
  }
}

template <int EQ>
__device__ __forceinline__ void point_flux(const double* U, int d, const Stage2D& P, double* f) {
  if constexpr (EQ == EQ_EULER) {
    if (d == 0) euler_flux2d_x(U, P.gam, f);
    else euler_flux2d_y(U, P.gam, f);
  } else {
    f[0] = scalar_flux<EQ>(U[0], d == 0 ? P.adv0 : P.adv1);
  }
}

// Twice the Lax-Friedrichs flux, f(u-) + f(u+) - alpha (u+ - u-), at one face point (the
// factor 1/2 is applied with the quadrature weight)
template <int EQ>
__device__ __forceinline__ void lf_flux2(const double* um, const double* up, int d, double alpha,
                                         const Stage2D& P, double* F) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  double fm[NC], fp[NC];
  point_flux<EQ>(um, d, P, fm);
  point_flux<EQ>(up, d, P, fp);
#pragma unroll
  for (int c = 0; c < NC; ++c) F[c] = fma(-alpha, up[c] - um[c], fm[c] + fp[c]);
}

template <int EQ, int NGE, int BK>
__global__ __launch_bounds__(NT, NGE == 2 ? 3 : 2) void stage2d_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int NF = 3 * NC;
  __shared__ double s_u[NF * NP2];   // stage input, limited, on tile+2
  __shared__ double s_ring[2 * 2 * TX * NC * NGE];          // ring cells' face values
  __shared__ double s_bnd[(NT / 64) * 2 * TX * NC * NGE];   // y faces between waves
  __shared__ uint8_t s_T[NP2];
  __shared__ uint8_t s_H[NP2];
  __shared__ double s_red[8];
  __shared__ double s_alpha[2];

  const int mode = P.mode;
  // the time step (zero once the run has reached its final time: nothing to do) is
  // checked after the stage input's loads are issued
  const double dtv = *P.dt;   // (valid in every mode)
  const double dt = mode != MODE_L ? dtv : 0.0;
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - H2, gy0 = by * TY - H2;
  const size_t plane = (size_t)nx * ny;
  const bool tc = P.tc_mode != TC_NONE;

  // ---------------------------------------------------------------- stage input -> LDS
  // flagged cells take the prepass's limited first moments; ghosts mirror their cell
  // each thread's (at most NR) positions: flags and stored values are loaded first, the
  // limited moments of the (few) flagged cells replace the moments afterwards
  constexpr int NR = (NP2 + NT - 1) / NT;
  size_t gsr[NR];
  double sxr[NR], syr[NR];
  uint8_t tr[NR], hr[NR];
  uint8_t fwr[NR];   // forward step: bit 0 rho u, bit 1 rho v reversed
  double v[NR][NF];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = tid + r * NT;
    tr[r] = 0;
    hr[r] = 0;
    fwr[r] = 0;
    if (q < NP2) {
      const int ly = q / L2, lx = q - ly * L2;
      int gx, gy;
      if constexpr (BK == BK_STEP) {
        const step::Src sr = step::resolve(gx0 + lx, gy0 + ly, nx, ny, P.si, P.sj);
        gx = sr.x;
        gy = sr.y;
        sxr[r] = sr.sx;
        syr[r] = sr.sy;
        fwr[r] = (sr.fu < 0.0 ? 1 : 0) | (sr.fv < 0.0 ? 2 : 0);
        if (sr.pres) {
          // inflow: the prescribed state, zero first moments, never troubled
          gsr[r] = 0;
#pragma unroll
          for (int f = 0; f < NF; ++f) v[r][f] = f < NC ? P.uin[f] : 0.0;
          continue;
        }
      } else {
        gx = map_index(gx0 + lx, nx, P.bcx, sxr[r]);
        gy = map_index(gy0 + ly, ny, P.bcy, syr[r]);
      }
      gsr[r] = (size_t)gy * nx + gx;
      if (dmr_prescribed<BK>(P, gx0 + lx, gy0 + ly)) {
        // prescribed ghost: the exact solution, never troubled, no mirror signs
        const double ts = stage_time_of<BK>(P, dtv);
#pragma unroll
        for (int f = 0; f < NF; ++f) v[r][f] = dmr_value(P, f, gx0 + lx, gy0 + ly, ts);
        sxr[r] = syr[r] = 1.0;
        continue;
      }
      if (tc) {
        tr[r] = P.Tcur[gsr[r]];
        hr[r] = P.Hcur[gsr[r]];   // a ghost's mask is that of the cell it mirrors
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) v[r][f] = P.in[f * plane + gsr[r]];
    }
  }
  if (mode != MODE_L && dt == 0.0) return;   // uniform over the grid
  // this stage's prepasses are done: record the list lengths, empty the lists for the next
  // stage
  if (tc && blockIdx.x == 0 && tid == 0) {
    const int st = mode == MODE_L ? 0 : mode - MODE_RK1;
    P.stats[st] = P.counts[0];
    P.stats[3 + st] = P.counts[1];
    P.counts[0] = 0;
    P.counts[1] = 0;
  }
  reduce_speeds(P.alpha_in, s_alpha);   // visible after the staging barrier
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = tid + r * NT;
    if (q < NP2) {
      if (tr[r]) {
#pragma unroll
        for (int f = NC; f < NF; ++f) v[r][f] = P.limcur[(f - NC) * plane + gsr[r]];
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int m = f / NC, c = f % NC;
        double wf;
        if constexpr (BK == BK_STEP) wf = ((c == 1 && (fwr[r] & 1)) || (c == 2 && (fwr[r] & 2))) ? -1.0 : 1.0;
        else wf = wall_factor<EQ>(c, sxr[r] < 0.0, syr[r] < 0.0, P.bcx, P.bcy);
        s_u[f * NP2 + q] = wf * (m == 1 ? sxr[r] * v[r][f] : (m == 2 ? syr[r] * v[r][f] : v[r][f]));
      }
      s_T[q] = tr[r];
      s_H[q] = hr[r];
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- tile cell
  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + H2, ly = ty + H2;
  const int gx = gx0 + lx, gy = gy0 + ly;
  const bool inmesh = gx < nx && gy < ny;
  // the solid cells of the forward step are never updated
  bool active = inmesh;
  if constexpr (BK == BK_STEP) active = inmesh && !step::solid(gx, gy, P.si, P.sj);

  const int lane = tid & 63, wv = tid >> 6;
  // stages 2 and 3: whether u^n of this cell was limited (read now, so that the epilogue
  // issues the loads of u^n and of its limited moments together)
  const bool rk23 = mode == MODE_RK2 || mode == MODE_RK3;
  const uint8_t tn = (rk23 && active) ? P.Tn[(size_t)gy * nx + gx] : 0;
  // ring cells (the tile's neighbours across its four sides), all 64 by wave 0: lanes
  // 32 d .. 32 d + 31 those of direction d, the low side's high-face values and the high
  // side's low-face values
  if (wv == 0) {
    const int rd = lane / (2 * TX), rs = (lane / TX) & 1, rp = lane % TX;
    const int rly = rd == 0 ? H2 + rp : (rs == 0 ? H2 - 1 : H2 + TY);
    const int rlx = rd == 0 ? (rs == 0 ? H2 - 1 : H2 + TX) : H2 + rp;
    double a[NC][NGE], b[NC][NGE];
    cell_traces<EQ, NGE, -1, BK>(P, s_u, s_H[rly * L2 + rlx] != 0, rly, rlx, rd, gx0, gy0, a, b);
    if constexpr (BK == BK_DMR) {
      if (dmr_prescribed<BK>(P, gx0 + rlx, gy0 + rly)) {
        // the face shared with the tile: the ring cell's high face (rs = 0) or low face
        const double ts = stage_time_of<BK>(P, dtv);
        const int gxr = gx0 + rlx, gyr = gy0 + rly;
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          const double e = Gauss<NGE>::node[k];
          double x, y, U[4];
          if (rd == 0) {
            x = P.x0 + (gxr + (rs == 0 ? 1.0 : 0.0)) * P.dx;
            y = P.y0 + (gyr + 0.5 + e) * P.dy;
          } else {
            x = P.x0 + (gxr + 0.5 + e) * P.dx;
            y = P.y0 + (gyr + (rs == 0 ? 1.0 : 0.0)) * P.dy;
          }
          dmr::point_state(x, y, ts, P.gam, U);
#pragma unroll
          for (int c = 0; c < NC; ++c) a[c][k] = b[c][k] = U[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int k = 0; k < NGE; ++k)
        s_ring[(((rd * 2 + rs) * NC + c) * NGE + k) * TX + rp] = rs == 0 ? b[c][k] : a[c][k];
  }
  double RU[NC], RV[NC], RW[NC];
  // volume quadrature: (1/dx) sum w_k w_l f(u(G_kl)) and (1/dy) sum w_k w_l g(u(G_kl))
  {
    double inner[NC][9];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19];
      gather19<NC, L2>(s_u, c, ly, lx, in);
      hw2::lin2d_inner(in, inner[c]);
      __builtin_amdgcn_sched_barrier(0);
    }
    double sf[NC], sg[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) sf[c] = sg[c] = 0.0;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const double wq = VW[p % 3] * VW[p / 3];
      double U[NC], f[NC], g[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) U[c] = inner[c][p];
      if constexpr (EQ == EQ_EULER) {
        euler_flux2d_xy(U, P.gam, f, g);
      } else {
        f[0] = scalar_flux<EQ>(U[0], P.adv0);
        g[0] = scalar_flux<EQ>(U[0], P.adv1);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sf[c] = fma(wq, f[c], sf[c]);
        sg[c] = fma(wq, g[c], sg[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      RU[c] = 0.0;
      RV[c] = sf[c] * P.idx;
      RW[c] = sg[c] * P.idy;
    }
  }

  const double* node = Gauss<NGE>::node;
  const double* wt = Gauss<NGE>::wt;
#pragma unroll 1
  for (int dir = 0; dir < 2; ++dir) {
    // edge values: this cell's two sides; the low neighbour's high side and the high
    // neighbour's low side come from the lanes that own those cells (x: the next lane of
    // the 16-lane row; y: 16 lanes away, or the neighbouring wave's row through LDS), and
    // across the tile's sides from the ring values
    double ol[NC][NGE], oh[NC][NGE];
    const bool hyb = s_H[ly * L2 + lx] != 0;
    if (dir == 0) cell_traces<EQ, NGE, 0, BK>(P, s_u, hyb, ly, lx, 0, gx0, gy0, ol, oh);
    else cell_traces<EQ, NGE, 1, BK>(P, s_u, hyb, ly, lx, 1, gx0, gy0, ol, oh);
    const bool edge_lo = dir == 0 ? tx == 0 : (ty & 3) == 0;
    const bool edge_hi = dir == 0 ? tx == TX - 1 : (ty & 3) == 3;
    if (dir == 1) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          if (edge_lo) s_bnd[(((wv * 2 + 0) * NC + c) * NGE + k) * TX + tx] = ol[c][k];
          if (edge_hi) s_bnd[(((wv * 2 + 1) * NC + c) * NGE + k) * TX + tx] = oh[c][k];
        }
    }
    __syncthreads();
    // where the neighbour's value is read from LDS (ring or neighbouring wave)
    const double* lo_src = nullptr;
    const double* hi_src = nullptr;
    if (dir == 0) {
      lo_src = s_ring + (0 * 2 + 0) * NC * NGE * TX + ty;
      hi_src = s_ring + (0 * 2 + 1) * NC * NGE * TX + ty;
    } else {
      lo_src = wv == 0 ? s_ring + (1 * 2 + 0) * NC * NGE * TX + tx
                       : s_bnd + ((wv - 1) * 2 + 1) * NC * NGE * TX + tx;
      hi_src = wv == NT / 64 - 1 ? s_ring + (1 * 2 + 1) * NC * NGE * TX + tx
                                 : s_bnd + ((wv + 1) * 2 + 0) * NC * NGE * TX + tx;
    }
    const int step = dir == 0 ? 1 : TX;
    const int from_lo = (lane - step) & 63, from_hi = (lane + step) & 63;
    const double alpha = s_alpha[dir];
    const double inv = dir == 0 ? P.idx : P.idy;
    // face fluxes point by point, accumulated straight into the right-hand sides:
    // x faces feed the x moment with (F_L + F_R)/2 and the y moment with the node-weighted
    // difference, y faces the other way round
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      double um[NC], up[NC], FL[NC], FR[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double l = __shfl(oh[c][k], from_lo, 64);
        um[c] = edge_lo ? lo_src[(c * NGE + k) * TX] : l;
        up[c] = ol[c][k];
      }
      if constexpr (BK == BK_STEP) {
        // face rule: the inflow state on the left side; at the bottom wall and the step's
        // top face the cell's own trace with rho v reversed
        if (dir == 0 ? gx == 0 : (gy == 0 || (gy == P.sj && gx >= P.si))) {
#pragma unroll
          for (int c = 0; c < NC; ++c) um[c] = dir == 0 ? P.uin[c] : (c == 2 ? -ol[c][k] : ol[c][k]);
        }
      }
      lf_flux2<EQ>(um, up, dir, alpha, P, FL);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double r = __shfl(ol[c][k], from_hi, 64);
        um[c] = oh[c][k];
        up[c] = edge_hi ? hi_src[(c * NGE + k) * TX] : r;
      }
      if constexpr (BK == BK_STEP) {
        // face rule: the outflow takes the cell's own trace; the step's left face (rho u)
        // and the top wall (rho v) reverse the normal momentum
        if (dir == 0 ? (gx == nx - 1 || (gx == P.si - 1 && gy < P.sj)) : gy == ny - 1) {
          const int cn = dir == 0 ? (gx == nx - 1 ? -1 : 1) : 2;
#pragma unroll
          for (int c = 0; c < NC; ++c) up[c] = c == cn ? -oh[c][k] : oh[c][k];
        }
      }
      if constexpr (BK == BK_DMR) {
        // the top boundary: the prescribed ghost's trace is the exact state at the face's
        // Gauss points (the ring pass stores the same values; this also covers a ghost
        // that sits inside a partial last row of tiles)
        if (dir == 1 && gy == ny - 1) {
          double U[4];
          dmr::point_state(P.x0 + (gx + 0.5 + node[k]) * P.dx, P.y0 + ny * P.dy,
                           stage_time_of<BK>(P, dtv), P.gam, U);
#pragma unroll
          for (int c = 0; c < NC; ++c) up[c] = U[c];
        }
      }
      lf_flux2<EQ>(um, up, dir, alpha, P, FR);
      // FL, FR hold twice the fluxes
      const double wd = 0.5 * wt[k] * inv, wm = 0.5 * wt[k] * node[k] * inv;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        RU[c] = fma(-wd, FR[c] - FL[c], RU[c]);
        if (dir == 0) {
          RV[c] = fma(-0.5 * wd, FL[c] + FR[c], RV[c]);
          RW[c] = fma(-wm, FR[c] - FL[c], RW[c]);
        } else {
          RW[c] = fma(-0.5 * wd, FL[c] + FR[c], RW[c]);
          RV[c] = fma(-wm, FR[c] - FL[c], RV[c]);
        }
      }
    }
  }

  // ---------------------------------------------------------------- epilogue
  const uint8_t myT = s_T[ly * L2 + lx];
  double sp0 = 0.0, sp1 = 0.0;
  if constexpr (BK == BK_STEP) {
    // solid cells: no flags; the operator alone reports zero and the stored state
    if (inmesh && !active) {
      const size_t gi = (size_t)gy * nx + gx;
      if (P.flagsT) P.flagsT[gi] = 0;
      if (P.flagsH) P.flagsH[gi] = 0;
      if (mode == MODE_L) {
#pragma unroll
        for (int f = 0; f < NF; ++f) P.out[(size_t)f * plane + gi] = 0.0;
        if (P.wout) {
#pragma unroll
          for (int f = 0; f < NF; ++f) P.wout[(size_t)f * plane + gi] = P.in[(size_t)f * plane + gi];
        }
      }
    }
  }
  if (active) {
    const size_t gi = (size_t)gy * nx + gx;
    if (P.flagsT) P.flagsT[gi] = myT;
    if (P.flagsH) P.flagsH[gi] = s_H[ly * L2 + lx];
    double own[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) own[f] = S<L2>(s_u, f, ly, lx);   // limited stage input
    if (mode == MODE_L) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        P.out[(size_t)c * plane + gi] = RU[c];
        P.out[(size_t)(NC + c) * plane + gi] = RV[c];
        P.out[(size_t)(2 * NC + c) * plane + gi] = RW[c];
      }
      if (P.wout) {
#pragma unroll
        for (int f = 0; f < NF; ++f) P.wout[(size_t)f * plane + gi] = own[f];
      }
    } else {
      double Wn[NF];
      if (mode == MODE_RK1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) Wn[f] = own[f];
      } else {
#pragma unroll
        for (int f = 0; f < NC; ++f) Wn[f] = P.base[(size_t)f * plane + gi];
        if (tn) {
#pragma unroll
          for (int f = NC; f < NF; ++f) Wn[f] = P.limn[(size_t)(f - NC) * plane + gi];
        } else {
#pragma unroll
          for (int f = NC; f < NF; ++f) Wn[f] = P.base[(size_t)f * plane + gi];
        }
      }
      // out = a W(u^n) + b (W(u^(s)) + dt L), with (a, b) of the stage (eq. RK)
      double ca, cb;
      rk_coeffs(mode, ca, cb);
      const double cdt = cb * dt;
      double res[NF];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double L3[3] = {RU[c], RV[c], RW[c]};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int f = m * NC + c;
          res[f] = fma(cdt, L3[m], fma(ca, Wn[f], cb * own[f]));
        }
      }
      int bad = 0;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        P.out[(size_t)f * plane + gi] = res[f];
        if (!isfinite(res[f])) bad |= 1;
      }
      if constexpr (EQ == EQ_EULER) {
        double p;
        euler_speeds2d(res, P.gam, sp0, sp1, p);
        if (!(res[0] > 0.0) || !(p > 0.0)) bad |= 2;
      } else if constexpr (EQ == EQ_BURGERS) {
        sp0 = sp1 = fabs(res[0]);
      } else {
        sp0 = fabs(P.adv0);
        sp1 = fabs(P.adv1);
      }
      if (bad) atomicOr(P.status, bad);
    }
  }
  if (mode != MODE_L) {
    // block maxima of both directions with one barrier
    const double w0 = wave_max(sp0), w1 = wave_max(sp1);
    if (lane == 0) {
      s_red[wv] = w0;
      s_red[4 + wv] = w1;
    }
    __syncthreads();
    if (tid == 0) {
      const double m0 = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
      const double m1 = fmax(fmax(s_red[4], s_red[5]), fmax(s_red[6], s_red[7]));
      const int e = blockIdx.x % ASPREAD;
      atomic_max_pos(&P.alpha_out[e], m0);
      atomic_max_pos(&P.alpha_out[ASPREAD + e], m1);
    }
  }
}

// Lax-Friedrichs speeds of a state (used before the first stage and by the operator-only
// entry point): per-direction max over cells of the spectral radius at the averages.
template <int EQ>
__global__ __launch_bounds__(256) void alpha2d_kernel(const double* U, int nx, int ny, double gam,
                                                      double a0, double a1, int si, int sj,
                                                      unsigned long long* alpha_out) {
  __shared__ double s_red[4];
  const size_t plane = (size_t)nx * ny;
  double m0 = 0.0, m1 = 0.0;
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < plane; i += (size_t)gridDim.x * 256) {
    if (si < nx) {
      // the solid cells of the forward step hold no flow
      const size_t gy = i / nx;
      if ((int)(i - gy * nx) >= si && (int)gy < sj) continue;
    }
    if constexpr (EQ == EQ_EULER) {
      double Ub[4], s0, s1, p;
      for (int c = 0; c < 4; ++c) Ub[c] = U[c * plane + i];
      euler_speeds2d(Ub, gam, s0, s1, p);
      m0 = fmax(m0, s0);
      m1 = fmax(m1, s1);
    } else if constexpr (EQ == EQ_BURGERS) {
      m0 = fmax(m0, fabs(U[i]));
      m1 = m0;
    } else {
      m0 = fabs(a0);
      m1 = fabs(a1);
    }
  }
  const double r0 = block_max256(m0, s_red);
  __syncthreads();
  const double r1 = block_max256(m1, s_red);
  if (threadIdx.x == 0) {
    const int e = blockIdx.x % ASPREAD;
    atomic_max_pos(&alpha_out[e], r0);
    atomic_max_pos(&alpha_out[ASPREAD + e], r1);
  }
}

// The double Mach reflection's prescribed ghost cells at the stage's time: the cut-cell
// moments of the exact solution (hw_dmr.h) at every position of the two ghost layers that
// is prescribed, one thread per (position, field); the stage's four kernels read them.
__global__ __launch_bounds__(NT) void dmr_table_kernel(Stage2D P) {
  constexpr int NF = 12;
  const double dtv = *P.dt;
  if (P.mode != MODE_L && dtv == 0.0) return;   // the run has reached its final time
  const double ts = dmr::stage_time(P.t, dtv, P.mode);
  const int nx = P.nx, ny = P.ny, nr = dmr::ring2_size(nx, ny);
  for (int q = blockIdx.x * NT + threadIdx.x; q < NF * nr; q += gridDim.x * NT) {
    const int f = q / nr, r = q - f * nr;
    int gx, gy;
    dmr::ring2_position(r, nx, ny, gx, gy);
    P.dtab[q] = dmr::prescribed(gx, gy, nx, ny, P.x0, P.dx)
                    ? dmr::cell_value(f, P.x0 + (gx + 0.5) * P.dx, P.y0 + (gy + 0.5) * P.dy, P.dx, ts, P.gam)
                    : 0.0;
  }
}

}  // namespace hw

// ------------------------------------------------------------------ launch wrappers
extern "C" hipError_t hw_launch_stage2d(int eq, int ng, const hw::Stage2D* P, hipStream_t s,
                                        hipEvent_t* ev) {
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 block(hw::NT);
  const bool pre = P->tc_mode != hw::TC_NONE;
  // work-list passes: a grid of a few workgroups per compute unit strides over the items
  const int wgrid = 2048;
#define HW_MARK(i) \
  if (ev && hipEventRecord(ev[i], s) != hipSuccess) return hipErrorLaunchFailure
#define HW_L2(E, G, D)                                                                  \
  do {                                                                                  \
    if (pre) hipLaunchKernelGGL((hw::stage2d_flags_kernel<E, D>), grid, block, 0, s, *P); \
    HW_MARK(0);                                                                         \
    if (pre) hipLaunchKernelGGL((hw::stage2d_limit_kernel<E, D>), dim3(wgrid), block, 0, s, *P); \
    HW_MARK(1);                                                                         \
    if (pre) hipLaunchKernelGGL((hw::stage2d_hweno_kernel<E, G, D>), dim3(wgrid), block, 0, s, *P); \
    HW_MARK(2);                                                                         \
    hipLaunchKernelGGL((hw::stage2d_kernel<E, G, D>), grid, block, 0, s, *P);           \
  } while (0)
  // the double Mach reflection and forward-step boundaries (Euler only) have kernel
  // instances of their own
  const int bk = P->bcx == hw::BC_DMR ? hw::BK_DMR : (P->bcx == hw::BC_STEP ? hw::BK_STEP : hw::BK_RECT);
  if (bk != hw::BK_RECT && eq != hw::EQ_EULER) return hipErrorInvalidValue;
  if (bk == hw::BK_DMR) {
    if (!P->dtab) return hipErrorInvalidValue;
    const int nq = 12 * (4 * (P->nx + 4) + 4 * P->ny);
    hipLaunchKernelGGL(hw::dmr_table_kernel, dim3((nq + hw::NT - 1) / hw::NT), block, 0, s, *P);
  }
  if (eq == hw::EQ_EULER && ng == 2 && bk == hw::BK_DMR) HW_L2(hw::EQ_EULER, 2, hw::BK_DMR);
  else if (eq == hw::EQ_EULER && ng == 3 && bk == hw::BK_DMR) HW_L2(hw::EQ_EULER, 3, hw::BK_DMR);
  else if (eq == hw::EQ_EULER && ng == 2 && bk == hw::BK_STEP) HW_L2(hw::EQ_EULER, 2, hw::BK_STEP);
  else if (eq == hw::EQ_EULER && ng == 3 && bk == hw::BK_STEP) HW_L2(hw::EQ_EULER, 3, hw::BK_STEP);
  else if (eq == hw::EQ_EULER && ng == 2) HW_L2(hw::EQ_EULER, 2, hw::BK_RECT);
  else if (eq == hw::EQ_EULER && ng == 3) HW_L2(hw::EQ_EULER, 3, hw::BK_RECT);
  else if (eq == hw::EQ_BURGERS && ng == 2) HW_L2(hw::EQ_BURGERS, 2, hw::BK_RECT);
  else if (eq == hw::EQ_BURGERS && ng == 3) HW_L2(hw::EQ_BURGERS, 3, hw::BK_RECT);
  else if (eq == hw::EQ_ADV && ng == 2) HW_L2(hw::EQ_ADV, 2, hw::BK_RECT);
  else if (eq == hw::EQ_ADV && ng == 3) HW_L2(hw::EQ_ADV, 3, hw::BK_RECT);
  else return hipErrorInvalidValue;
#undef HW_L2
#undef HW_MARK
  return hipGetLastError();
}

// the forward prepasses alone (the reverse mode reruns them on a stored stage input): flags
// and work lists, the limiter, the HWENO edge values; rectangles with periodic, transmissive
// or reflective sides, and the forward step (si, sj, uin set)
extern "C" hipError_t hw_launch_prepass2d(int eq, int ng, const hw::Stage2D* P, hipStream_t s) {
  if (P->tc_mode == hw::TC_NONE) return hipSuccess;
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 block(hw::NT);
  const int wgrid = 2048;
#define HW_PP(E, G, B)                                                                         \
  do {                                                                                         \
    hipLaunchKernelGGL((hw::stage2d_flags_kernel<E, B>), grid, block, 0, s, *P);               \
    hipLaunchKernelGGL((hw::stage2d_limit_kernel<E, B>), dim3(wgrid), block, 0, s, *P);        \
    hipLaunchKernelGGL((hw::stage2d_hweno_kernel<E, G, B>), dim3(wgrid), block, 0, s, *P);     \
  } while (0)
  // rectangles with mirrored or periodic sides, and the forward step
  const bool step = P->bcx == hw::BC_STEP;
  // the double Mach reflection: its prescribed ghosts of the stage's time first (dtab)
  const bool dmrb = P->bcx == hw::BC_DMR;
  if (dmrb && eq == hw::EQ_EULER && (ng == 2 || ng == 3)) {
    if (!P->dtab) return hipErrorInvalidValue;
    const int nq = 12 * hw::dmr::ring2_size(P->nx, P->ny);
    hipLaunchKernelGGL(hw::dmr_table_kernel, dim3((nq + hw::NT - 1) / hw::NT), block, 0, s, *P);
  }
  if (eq == hw::EQ_EULER && ng == 2 && dmrb) HW_PP(hw::EQ_EULER, 2, hw::BK_DMR);
  else if (eq == hw::EQ_EULER && ng == 3 && dmrb) HW_PP(hw::EQ_EULER, 3, hw::BK_DMR);
  else if (eq == hw::EQ_EULER && ng == 2 && !step) HW_PP(hw::EQ_EULER, 2, hw::BK_RECT);
  else if (eq == hw::EQ_EULER && ng == 3 && !step) HW_PP(hw::EQ_EULER, 3, hw::BK_RECT);
  else if (eq == hw::EQ_EULER && ng == 2) HW_PP(hw::EQ_EULER, 2, hw::BK_STEP);
  else if (eq == hw::EQ_EULER && ng == 3) HW_PP(hw::EQ_EULER, 3, hw::BK_STEP);
  else return hipErrorInvalidValue;
#undef HW_PP
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_alpha2d(int eq, const double* U, int nx, int ny, double gam,
                                        double a0, double a1, int si, int sj,
                                        unsigned long long* alpha_out, hipStream_t s) {
  const size_t n = (size_t)nx * ny;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (eq == hw::EQ_EULER)
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_EULER>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, si, sj, alpha_out);
  else if (eq == hw::EQ_BURGERS)
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_BURGERS>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, si, sj, alpha_out);
  else
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_ADV>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, si, sj, alpha_out);
  return hipGetLastError();
}

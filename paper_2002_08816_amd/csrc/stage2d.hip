// Two-dimensional stage of the hybrid Hermite WENO scheme (Zhao & Qiu, arXiv 2002.08816,
// Section 2.2, Steps 4-6 and eq. ode2), as two launches per Runge-Kutta stage:
//
//  stage2d_pre   (only when troubled cells are detected) per 16 x 16 tile with two ghost
//                layers: KXRCF flags (Step 4, Remark 3) and the Jacobi limiter of the first
//                moments (Step 4, Remark 4) on tile+1, the hybrid mask of the tile, and
//                the HWENO edge values (Step 5.1) of its hybrid cells.  The HWENO work is
//                spread one (cell, direction, characteristic field) per thread, so a tile
//                with a handful of hybrid cells finishes in one short pass.  Writes the
//                flags, the limited first moments of flagged cells and the hybrid cells'
//                edge values.
//  stage2d_main  per 16 x 16 tile with two ghost layers (flags and limited moments read
//                back): hybrid mask on tile+1, interior Gauss values of the least-squares
//                quartic -> volume integrals (Step 5.3); per direction, the edge values of
//                the cell and of its two neighbours (Step 5.2 linear, or the stored HWENO
//                values), the Lax-Friedrichs fluxes of its two faces and the edge
//                quadratures of eq. ode2; the TVD-RK3 stage combination (eq. RK) with the
//                limited moments, the store, and the block's share of the next stage's
//                speeds.  No data is exchanged between threads after staging: each face's
//                flux is evaluated by both of its cells from the same values.
//
// The limited first moments of the stage input replace the stored ones in the stage
// combination; the flags and limited moments of u^n (stage 1) are kept for stages 2, 3.
// Transmissive ghost cells are mirror images of the cells they copy in every respect
// (state, flag, limited moments, edge values).
#include "hw_tile2d.h"

namespace hw {

// ------------------------------------------------------------------ prepass
// distance-1 transmissive ghost positions of tile+1 take flags / limited state from the
// cell they mirror (ghost rows and columns are distinct from the cells they copy)
__device__ __forceinline__ int mirror1(int g, int n, int bc) {
  if (bc != BC_TRANSMISSIVE) return g;
  if (g == -1) return 0;
  if (g == n) return n - 1;
  return g;
}

template <int EQ, int NGE>
__global__ __launch_bounds__(NT) void stage2d_pre_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int NF = 3 * NC;
  __shared__ double s_in[NF * NPOS];       // stage input on tile+2, then limited on tile+1
  __shared__ uint8_t s_T[NPOS];
  __shared__ uint8_t s_H[NPOS];
  __shared__ short s_list[NT];
  __shared__ int s_count;
  __shared__ double s_v[NT * 2 * NGE];     // one HWENO item's edge values per thread

  if (P.mode != MODE_L && *P.dt == 0.0) return;   // the run has reached its final time
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - HL, gy0 = by * TY - HL;
  const size_t plane = (size_t)nx * ny;

  load_tile<NF, NC>(P.in, nx, ny, P.bcx, P.bcy, gx0, gy0, 1, s_in);
  if (tid == 0) s_count = 0;
  __syncthreads();
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T, 2);
  __syncthreads();
  const bool mir = P.bcx == BC_TRANSMISSIVE || P.bcy == BC_TRANSMISSIVE;
  constexpr int W1 = LX - 4;   // tile+1
  if (mir) {
    for (int q = tid; q < W1 * W1; q += NT) {
      const int ly = 2 + q / W1, lx = 2 + q % W1;
      const int mx = mirror1(gx0 + lx, nx, P.bcx) - gx0, my = mirror1(gy0 + ly, ny, P.bcy) - gy0;
      if (mx != lx || my != ly) s_T[ly * LX + lx] = s_T[my * LX + mx];
    }
    __syncthreads();
  }
  limit_tile<EQ>(s_in, s_T, P.gam, P.w, 2);
  if (mir) {
    __syncthreads();
    for (int q = tid; q < W1 * W1; q += NT) {
      const int ly = 2 + q / W1, lx = 2 + q % W1;
      const int gmx = mirror1(gx0 + lx, nx, P.bcx), gmy = mirror1(gy0 + ly, ny, P.bcy);
      const int mx = gmx - gx0, my = gmy - gy0;
      if (mx == lx && my == ly) continue;
      const double sx = mx != lx ? -1.0 : 1.0, sy = my != ly ? -1.0 : 1.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        s_in[((NC + c) * LY + ly) * LX + lx] = sx * s_in[((NC + c) * LY + my) * LX + mx];
        s_in[((2 * NC + c) * LY + ly) * LX + lx] = sy * s_in[((2 * NC + c) * LY + my) * LX + mx];
      }
    }
  }
  hybrid_tile(s_T, s_H, 3);
  __syncthreads();

  // this tile's flags and limited moments; hybrid cells into the work list
  {
    const int tx = tid % TX, ty = tid / TX;
    const int lx = tx + HL, ly = ty + HL;
    const int gx = gx0 + lx, gy = gy0 + ly;
    if (gx < nx && gy < ny) {
      const size_t gi = (size_t)gy * nx + gx;
      const uint8_t t = s_T[ly * LX + lx];
      P.Tcur[gi] = t;
      if (t) {
#pragma unroll
        for (int f = NC; f < NF; ++f) P.limcur[(size_t)(f - NC) * plane + gi] = S(s_in, f, ly, lx);
      }
      if (s_H[ly * LX + lx]) s_list[atomicAdd(&s_count, 1)] = (short)tid;
    }
  }
  __syncthreads();
  const int count = s_count;
  const int items = count * 2 * NC;
  // item = ((cell, direction), characteristic field), the field fastest
  for (int r0 = 0; r0 < items; r0 += NT) {
    const int it = r0 + tid;
    if (it < items) {
      const int f = it % NC, cd = it / NC, dir = cd & 1, cell = s_list[cd >> 1];
      const int ly = cell / TX + HL, lx = cell % TX + HL;
      double w19[19];
      if constexpr (EQ == EQ_EULER) {
        double U[4], Lr[4], Rc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) U[c] = S(s_in, c, ly, lx);
        euler_eig2d_field(U, P.gam, dir, f, Lr, Rc);
#pragma unroll
        for (int k = 0; k < 19; ++k) w19[k] = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double in[19];
          gather19<4>(s_in, c, ly, lx, in);
#pragma unroll
          for (int k = 0; k < 19; ++k) w19[k] = fma(Lr[c], in[k], w19[k]);
        }
      } else {
        gather19<1>(s_in, 0, ly, lx, w19);
      }
      double v[2 * NGE];
      hweno2d_field<NGE>(w19, P.w, dir, v);
#pragma unroll
      for (int k = 0; k < 2 * NGE; ++k) s_v[tid * 2 * NGE + k] = v[k];
    }
    __syncthreads();
    // back to conserved components: one thread per (cell, direction) of this round
    const int cd = r0 / NC + tid;
    if (tid < NT / NC && cd < count * 2) {
      const int dir = cd & 1, cell = s_list[cd >> 1];
      const int ly = cell / TX + HL, lx = cell % TX + HL;
      const size_t gi = (size_t)(gy0 + ly) * nx + (gx0 + lx);
      const double* vb = s_v + (size_t)tid * NC * 2 * NGE;
      double out[NC][2 * NGE];
      if constexpr (EQ == EQ_EULER) {
        double U[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) U[c] = S(s_in, c, ly, lx);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int k = 0; k < 2 * NGE; ++k) out[c][k] = 0.0;
#pragma unroll 1
        for (int f = 0; f < 4; ++f) {
          double Lr[4], Rc[4];
          euler_eig2d_field(U, P.gam, dir, f, Lr, Rc);
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 2 * NGE; ++k) out[c][k] = fma(Rc[c], vb[f * 2 * NGE + k], out[c][k]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 2 * NGE; ++k) out[0][k] = vb[k];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          P.G[((((size_t)(dir * 2 + 0) * NGE + k) * NC + c)) * plane + gi] = out[c][k];
          P.G[((((size_t)(dir * 2 + 1) * NGE + k) * NC + c)) * plane + gi] = out[c][NGE + k];
        }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ main stage kernel
constexpr int H2 = 2, L2 = TX + 2 * H2, NP2 = L2 * L2;   // tile + two ghost layers

// Edge values of the cell at LDS position (ly, lx) on the faces of direction dir (lo:
// left or bottom, hi: right or top; either may be null): p0 at the edge Gauss points
// (Step 5.2), or for a hybrid cell the values the prepass stored (Step 5.1).  A ghost's
// stored values are those of the cell it mirrors, faces and edge points reflected.
template <int EQ, int NGE>
__device__ __forceinline__ void cell_traces(const Stage2D& P, const double* s_u, bool hyb, int ly,
                                            int lx, int dir, int gx0, int gy0, double (*lo)[NGE],
                                            double (*hi)[NGE]) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  if (!hyb) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19], a[NGE], b[NGE];
      gather19<NC, L2>(s_u, c, ly, lx, in);
      lin_edges<NGE>(in, dir, a, b);
#pragma unroll
      for (int k = 0; k < NGE; ++k) {
        if (lo) lo[c][k] = a[k];
        if (hi) hi[c][k] = b[k];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  double sx, sy;
  const int gx = map_index(gx0 + lx, P.nx, P.bcx, sx);
  const int gy = map_index(gy0 + ly, P.ny, P.bcy, sy);
  const bool mx = sx < 0.0, my = sy < 0.0;
  const bool swap = dir == 0 ? mx : my, flip = dir == 0 ? my : mx;
  const size_t plane = (size_t)P.nx * P.ny, gi = (size_t)gy * P.nx + gx;
  const int slo = swap ? 1 : 0, shi = 1 - slo;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      const int kk = flip ? NGE - 1 - k : k;
      if (lo) lo[c][k] = P.G[((((size_t)(dir * 2 + slo) * NGE + kk) * NC + c)) * plane + gi];
      if (hi) hi[c][k] = P.G[((((size_t)(dir * 2 + shi) * NGE + kk) * NC + c)) * plane + gi];
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

// Lax-Friedrichs flux (f(u-) + f(u+))/2 - alpha (u+ - u-)/2 at one face point
template <int EQ>
__device__ __forceinline__ void lf_flux(const double* um, const double* up, int d, double alpha,
                                        const Stage2D& P, double* F) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  double fm[NC], fp[NC];
  point_flux<EQ>(um, d, P, fm);
  point_flux<EQ>(up, d, P, fp);
#pragma unroll
  for (int c = 0; c < NC; ++c) F[c] = 0.5 * (fm[c] + fp[c]) - 0.5 * alpha * (up[c] - um[c]);
}

template <int EQ, int NGE>
__global__ __launch_bounds__(NT, 2) void stage2d_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int NF = 3 * NC;
  __shared__ double s_u[NF * NP2];   // stage input, limited, on tile+2
  __shared__ uint8_t s_T[NP2];
  __shared__ uint8_t s_H[NP2];
  __shared__ double s_red[4];

  const int mode = P.mode;
  double dt = 0.0;
  if (mode != MODE_L) {
    dt = *P.dt;
    if (dt == 0.0) return;   // the run has reached its final time: nothing to do
  }
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - H2, gy0 = by * TY - H2;
  const size_t plane = (size_t)nx * ny;
  const bool tc = P.tc_mode != TC_NONE;

  // ---------------------------------------------------------------- stage input -> LDS
  // flagged cells take the prepass's limited first moments; ghosts mirror their cell
  for (int q = tid; q < NP2; q += NT) {
    const int ly = q / L2, lx = q - ly * L2;
    double sx, sy;
    const int gx = map_index(gx0 + lx, nx, P.bcx, sx);
    const int gy = map_index(gy0 + ly, ny, P.bcy, sy);
    const size_t gs = (size_t)gy * nx + gx;
    const uint8_t t = tc ? P.Tcur[gs] : 0;
    double v[NF];
#pragma unroll
    for (int f = 0; f < NC; ++f) v[f] = P.in[f * plane + gs];
    if (t) {
#pragma unroll
      for (int f = NC; f < NF; ++f) v[f] = P.limcur[(f - NC) * plane + gs];
    } else {
#pragma unroll
      for (int f = NC; f < NF; ++f) v[f] = P.in[f * plane + gs];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int m = f / NC;
      s_u[f * NP2 + q] = m == 1 ? sx * v[f] : (m == 2 ? sy * v[f] : v[f]);
    }
    s_T[q] = t;
  }
  __syncthreads();
  // hybrid mask on tile+1 (positions [1, L2 - 1))
  constexpr int W1 = L2 - 2;
  for (int q = tid; q < W1 * W1; q += NT) {
    const int ly = 1 + q / W1, lx = 1 + q % W1;
    uint8_t hm = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) hm |= s_T[(ly + dy) * L2 + lx + dx];
    s_H[ly * L2 + lx] = hm;
  }
  __syncthreads();

  // ---------------------------------------------------------------- tile cell
  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + H2, ly = ty + H2;
  const int gx = gx0 + lx, gy = gy0 + ly;
  const bool active = gx < nx && gy < ny;

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
      RV[c] = sf[c] / P.dx;
      RW[c] = sg[c] / P.dy;
    }
  }

  const double* node = Gauss<NGE>::node;
  const double* wt = Gauss<NGE>::wt;
#pragma unroll 1
  for (int dir = 0; dir < 2; ++dir) {
    const int oy = dir, ox = 1 - dir;
    // edge values: the low neighbour's high side, this cell's two sides, the high
    // neighbour's low side
    double tl[NC][NGE], ol[NC][NGE], oh[NC][NGE], tr[NC][NGE];
    cell_traces<EQ, NGE>(P, s_u, s_H[(ly - oy) * L2 + lx - ox] != 0, ly - oy, lx - ox, dir, gx0,
                         gy0, nullptr, tl);
    cell_traces<EQ, NGE>(P, s_u, s_H[ly * L2 + lx] != 0, ly, lx, dir, gx0, gy0, ol, oh);
    cell_traces<EQ, NGE>(P, s_u, s_H[(ly + oy) * L2 + lx + ox] != 0, ly + oy, lx + ox, dir, gx0,
                         gy0, tr, nullptr);
    const double alpha = __longlong_as_double((long long)P.alpha_in[dir]);
    const double inv = 1.0 / (dir == 0 ? P.dx : P.dy);
    double sdiff[NC], ssum[NC], smom[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) sdiff[c] = ssum[c] = smom[c] = 0.0;
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      double um[NC], up[NC], FL[NC], FR[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        um[c] = tl[c][k];
        up[c] = ol[c][k];
      }
      lf_flux<EQ>(um, up, dir, alpha, P, FL);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        um[c] = oh[c][k];
        up[c] = tr[c][k];
      }
      lf_flux<EQ>(um, up, dir, alpha, P, FR);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sdiff[c] = fma(wt[k], FR[c] - FL[c], sdiff[c]);
        ssum[c] = fma(wt[k], FL[c] + FR[c], ssum[c]);
        smom[c] = fma(wt[k] * node[k], FR[c] - FL[c], smom[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      RU[c] -= sdiff[c] * inv;
      if (dir == 0) {
        RV[c] -= 0.5 * ssum[c] * inv;
        RW[c] -= smom[c] * inv;
      } else {
        RV[c] -= smom[c] * inv;
        RW[c] -= 0.5 * ssum[c] * inv;
      }
    }
  }

  // ---------------------------------------------------------------- epilogue
  const uint8_t myT = s_T[ly * L2 + lx];
  double sp0 = 0.0, sp1 = 0.0;
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
        for (int f = 0; f < NF; ++f) Wn[f] = P.base[(size_t)f * plane + gi];
        if (P.Tn[gi]) {
#pragma unroll
          for (int f = NC; f < NF; ++f) Wn[f] = P.limn[(size_t)(f - NC) * plane + gi];
        }
      }
      double res[NF];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double L3[3] = {RU[c], RV[c], RW[c]};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int f = m * NC + c;
          double v;
          if (mode == MODE_RK1) v = own[f] + dt * L3[m];
          else if (mode == MODE_RK2) v = (0.75 * Wn[f] + 0.25 * own[f]) + (0.25 * dt) * L3[m];
          else v = (Wn[f] / 3.0 + (2.0 / 3.0) * own[f]) + ((2.0 / 3.0) * dt) * L3[m];
          res[f] = v;
        }
      }
      int bad = 0;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        P.out[(size_t)f * plane + gi] = res[f];
        if (!isfinite(res[f])) bad |= 1;
      }
      if constexpr (EQ == EQ_EULER) {
        const double p = euler_pressure2d(res, P.gam);
        if (!(res[0] > 0.0) || !(p > 0.0)) bad |= 2;
        sp0 = euler_speed2d(res, P.gam, 0);
        sp1 = euler_speed2d(res, P.gam, 1);
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
    const double m0 = block_max256(sp0, s_red);
    __syncthreads();
    const double m1 = block_max256(sp1, s_red);
    if (tid == 0) {
      atomic_max_pos(&P.alpha_out[0], m0);
      atomic_max_pos(&P.alpha_out[1], m1);
    }
  }
}

// Lax-Friedrichs speeds of a state (used before the first stage and by the operator-only
// entry point): per-direction max over cells of the spectral radius at the averages.
template <int EQ>
__global__ __launch_bounds__(256) void alpha2d_kernel(const double* U, int nx, int ny, double gam,
                                                      double a0, double a1,
                                                      unsigned long long* alpha_out) {
  __shared__ double s_red[4];
  const size_t plane = (size_t)nx * ny;
  double m0 = 0.0, m1 = 0.0;
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < plane; i += (size_t)gridDim.x * 256) {
    if constexpr (EQ == EQ_EULER) {
      double Ub[4];
      for (int c = 0; c < 4; ++c) Ub[c] = U[c * plane + i];
      m0 = fmax(m0, euler_speed2d(Ub, gam, 0));
      m1 = fmax(m1, euler_speed2d(Ub, gam, 1));
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
    atomic_max_pos(&alpha_out[0], r0);
    atomic_max_pos(&alpha_out[1], r1);
  }
}

}  // namespace hw

// ------------------------------------------------------------------ launch wrappers
extern "C" hipError_t hw_launch_stage2d(int eq, int ng, const hw::Stage2D* P, hipStream_t s) {
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 block(hw::NT);
  const bool pre = P->tc_mode != hw::TC_NONE;
#define HW_L2(E, G)                                                                     \
  do {                                                                                  \
    if (pre) hipLaunchKernelGGL((hw::stage2d_pre_kernel<E, G>), grid, block, 0, s, *P);  \
    hipLaunchKernelGGL((hw::stage2d_kernel<E, G>), grid, block, 0, s, *P);              \
  } while (0)
  if (eq == hw::EQ_EULER && ng == 2) HW_L2(hw::EQ_EULER, 2);
  else if (eq == hw::EQ_EULER && ng == 3) HW_L2(hw::EQ_EULER, 3);
  else if (eq == hw::EQ_BURGERS && ng == 2) HW_L2(hw::EQ_BURGERS, 2);
  else if (eq == hw::EQ_BURGERS && ng == 3) HW_L2(hw::EQ_BURGERS, 3);
  else if (eq == hw::EQ_ADV && ng == 2) HW_L2(hw::EQ_ADV, 2);
  else if (eq == hw::EQ_ADV && ng == 3) HW_L2(hw::EQ_ADV, 3);
  else return hipErrorInvalidValue;
#undef HW_L2
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_alpha2d(int eq, const double* U, int nx, int ny, double gam,
                                        double a0, double a1, unsigned long long* alpha_out,
                                        hipStream_t s) {
  const size_t n = (size_t)nx * ny;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (eq == hw::EQ_EULER)
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_EULER>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, alpha_out);
  else if (eq == hw::EQ_BURGERS)
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_BURGERS>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, alpha_out);
  else
    hipLaunchKernelGGL(hw::alpha2d_kernel<hw::EQ_ADV>, dim3(blocks), dim3(256), 0, s, U, nx, ny, gam, a0, a1, alpha_out);
  return hipGetLastError();
}

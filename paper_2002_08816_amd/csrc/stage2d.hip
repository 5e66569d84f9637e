// Fused two-dimensional stage kernel of the hybrid Hermite WENO scheme
// (Zhao & Qiu, arXiv 2002.08816, Section 2.2, Steps 4-6 and eq. ode2).
//
// One workgroup (256 threads, one per cell) owns a 16 x 16 tile.  The tile plus three
// ghost layers of the stage input is staged in LDS (boundary conditions applied on the
// fly) and stays there for the whole stage; then, without leaving the workgroup:
//   1. KXRCF flags on tile+2                     (Step 4, Remark 3)
//   2. limiter of the first moments on flagged cells, dimension by dimension,
//      characteristic-wise for Euler (Jacobi: all from unmodified data) (Step 4, Remark 4)
//   3. hybrid mask H = flag anywhere in the 3x3 block, on tile+1
//   4. interior Gauss values of the least-squares quartic -> volume integrals (Step 5.3)
//   5. per direction: edge values (Step 5.2 linear, Step 5.1 HWENO in H cells), one-sided
//      exchange through a small LDS buffer, one Lax-Friedrichs flux per face, edge
//      quadratures of eq. ode2
//   6. TVD-RK3 stage combination (eq. RK), store, and the block's share of the next
//      stage's Lax-Friedrichs speeds.
// Each phase re-reads its stencil from LDS, so only that phase's values occupy registers.
// The limited first moments of the stage input replace the stored ones in the stage
// combination; the limited moments of u^n computed in the first stage are kept (sparse,
// flagged cells only) for the second and third stages.
#include "hw_tile2d.h"

namespace hw {

// hybrid cells per HWENO round (bounded so that two workgroups fit a CU's LDS)
template <int NGE>
constexpr int hw_round() { return NGE == 2 ? 128 : 32; }

// Edge values of the cell at (ly, lx) on the two faces of direction dir (lo: left or
// bottom, hi: right or top): p0 (Step 5.2), or HWENO (Step 5.1) when hyb, for Euler in
// the characteristic fields of that direction at the cell average (Remark 4).
template <int EQ, int NGE>
__device__ __forceinline__ void cell_edges(const double* s, int ly, int lx, int dir, bool hyb,
                                           const Stage2D& P, double (*lo)[NGE], double (*hi)[NGE]) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  if (!hyb) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19];
      gather19<NC>(s, c, ly, lx, in);
      lin_edges<NGE>(in, dir, lo[c], hi[c]);
      // one component's stencil at a time in registers
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  if constexpr (EQ != EQ_EULER) {
    double in[19], v[2 * NGE];
    gather19<1>(s, 0, ly, lx, in);
    hweno2d_field<NGE>(in, P.w, dir, v);
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      lo[0][k] = v[k];
      hi[0][k] = v[NGE + k];
    }
  } else {
    double U[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c] = S(s, c, ly, lx);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < NGE; ++k) lo[c][k] = hi[c][k] = 0.0;
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      double Lr[4], Rc[4];
      euler_eig2d_field(U, P.gam, dir, f, Lr, Rc);
      double w19[19];
#pragma unroll
      for (int k = 0; k < 19; ++k) w19[k] = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double in[19];
        gather19<4>(s, c, ly, lx, in);
#pragma unroll
        for (int k = 0; k < 19; ++k) w19[k] = fma(Lr[c], in[k], w19[k]);
        __builtin_amdgcn_sched_barrier(0);
      }
      double v[2 * NGE];
      hweno2d_field<NGE>(w19, P.w, dir, v);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          lo[c][k] = fma(Rc[c], v[k], lo[c][k]);
          hi[c][k] = fma(Rc[c], v[NGE + k], hi[c][k]);
        }
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

template <int EQ, int NGE>
__global__ __launch_bounds__(NT, 2) void stage2d_kernel(Stage2D P) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  constexpr int NF = 3 * NC;
  constexpr int NFACE = TX + 1;                 // faces per tile line
  __shared__ double s_in[NF * NPOS];
  __shared__ double s_x[NC * NGE * TY * NFACE]; // one-sided face exchange: trace, then flux
  __shared__ double s_x0[NC * NGE * TY];        // low ring's traces on face 0
  constexpr int HWK = hw_round<NGE>();
  __shared__ double s_hw[HWK * NC * NGE];       // HWENO high-face traces, one round
  __shared__ short s_list[NT + 2 * TY];         // hybrid cells of this direction
  __shared__ short s_slot[NT];                  // list slot of each tile cell (-1: none)
  __shared__ int s_count;
  __shared__ uint8_t s_T[NPOS];
  __shared__ uint8_t s_H[NPOS];
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
  const int gx0 = bx * TX - HL, gy0 = by * TY - HL;
  const size_t plane = (size_t)nx * ny;

  // ---------------------------------------------------------------- stage input -> LDS
  load_tile<NF, NC>(P.in, nx, ny, P.bcx, P.bcy, gx0, gy0, 0, s_in);
  __syncthreads();
  // ---------------------------------------------------------------- flags on tile+2
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T);
  __syncthreads();
  // ---------------------------------------------------------------- limiter (Jacobi)
  if (P.tc_mode != TC_NONE) limit_tile<EQ>(s_in, s_T, P.gam, P.w);
  // ---------------------------------------------------------------- hybrid mask, tile+1
  hybrid_tile(s_T, s_H);
  __syncthreads();

  // ---------------------------------------------------------------- tile cell
  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + HL, ly = ty + HL;
  const int gx = gx0 + lx, gy = gy0 + ly;
  const bool active = gx < nx && gy < ny;
  const bool hyb = s_H[ly * LX + lx] != 0;

  // right-hand-side accumulators (averages, x-moments, y-moments)
  double RU[NC], RV[NC], RW[NC];
  // volume quadrature: (1/dx) sum w_k w_l f(u(G_kl)) and (1/dy) sum w_k w_l g(u(G_kl))
  {
    double inner[NC][9];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19];
      gather19<NC>(s_in, c, ly, lx, in);
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

  // Ring cells: the 16 cells beyond each side of the tile supply the traces of the
  // tile's outer faces.  In direction dir, ring cell rr (0..31; rr < 16 on the low side)
  // is handled by lane rr % 8 of wave rr / 8, so every wave takes 8 of them.
  const int lane = tid & 63, wv = tid >> 6;
  const bool ring_thread = lane < 8;
  const int rr = wv * 8 + lane;
  const bool ring_low = rr < TY;
  const int rpos = rr % TY;

  const double* node = Gauss<NGE>::node;
  const double* wt = Gauss<NGE>::wt;
  auto xidx = [](int c, int k, int line, int face) {
    return ((c * NGE + k) * TY + line) * NFACE + face;
  };
#pragma unroll 1
  for (int dir = 0; dir < 2; ++dir) {
    const int line = dir == 0 ? ty : tx, pos = dir == 0 ? tx : ty;
    // linear traces first (Step 5.2), uniformly for every cell: ring cells publish theirs
    // (the high ring its low-face trace = u^+ of face 16, the low ring its high-face
    // trace = u^- of face 0, in s_x0); tile cells publish the low one (u^+ of face pos)
    // and keep the high one (u^- of face pos + 1)
    int rly = 0, rlx = 0;
    if (ring_thread) {
      rly = dir == 0 ? HL + rpos : (ring_low ? HL - 1 : HL + TY);
      rlx = dir == 0 ? (ring_low ? HL - 1 : HL + TX) : HL + rpos;
      double rlo[NC][NGE], rhi[NC][NGE];
      cell_edges<EQ, NGE>(s_in, rly, rlx, dir, false, P, rlo, rhi);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          if (ring_low) s_x0[(c * NGE + k) * TY + rpos] = rhi[c][k];
          else s_x[xidx(c, k, rpos, TX)] = rlo[c][k];
        }
    }
    double lo[NC][NGE], hi[NC][NGE];
    cell_edges<EQ, NGE>(s_in, ly, lx, dir, false, P, lo, hi);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int k = 0; k < NGE; ++k) s_x[xidx(c, k, line, pos)] = lo[c][k];
    // HWENO (Step 5.1) for the hybrid cells, compacted into a list so that the costly
    // branch runs on full waves: entries < NT are tile cells, NT + rr ring cells
    if (P.tc_mode != TC_NONE) {
      if (tid == 0) s_count = 0;
      s_slot[tid] = -1;
      __syncthreads();
      if (hyb) {
        const int k = atomicAdd(&s_count, 1);
        s_list[k] = (short)tid;
        s_slot[tid] = (short)k;
      }
      if (ring_thread && s_H[rly * LX + rlx]) s_list[atomicAdd(&s_count, 1)] = (short)(NT + rr);
      __syncthreads();
      const int count = s_count;
      for (int r0 = 0; r0 < count; r0 += HWK) {
        const int e = r0 + tid;
        if (tid < HWK && e < count) {
          const int id = s_list[e];
          int ely, elx, eline, epos, erp = 0;
          bool ering = id >= NT, elow = false;
          if (!ering) {
            const int etx = id % TX, ety = id / TX;
            elx = etx + HL; ely = ety + HL;
            eline = dir == 0 ? ety : etx;
            epos = dir == 0 ? etx : ety;
          } else {
            const int err = id - NT;
            elow = err < TY;
            erp = err % TY;
            ely = dir == 0 ? HL + erp : (elow ? HL - 1 : HL + TY);
            elx = dir == 0 ? (elow ? HL - 1 : HL + TX) : HL + erp;
            eline = erp;
            epos = 0;
          }
          double hlo[NC][NGE], hhi[NC][NGE];
          cell_edges<EQ, NGE>(s_in, ely, elx, dir, true, P, hlo, hhi);
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int k = 0; k < NGE; ++k) {
              if (!ering) {
                s_x[xidx(c, k, eline, epos)] = hlo[c][k];
                s_hw[(tid * NC + c) * NGE + k] = hhi[c][k];
              } else if (elow) {
                s_x0[(c * NGE + k) * TY + erp] = hhi[c][k];
              } else {
                s_x[xidx(c, k, erp, TX)] = hlo[c][k];
              }
            }
        }
        __syncthreads();
        const int sl = s_slot[tid];
        if (sl >= r0 && sl < r0 + HWK) {
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int k = 0; k < NGE; ++k) hi[c][k] = s_hw[((sl - r0) * NC + c) * NGE + k];
        }
        __syncthreads();
      }
    }
    __syncthreads();
    // Lax-Friedrichs flux on the high face (face pos + 1), and on face 0 by the low ring
    const double alpha = __longlong_as_double((long long)P.alpha_in[dir]);
    {
      double Fh[NC][NGE];
#pragma unroll
      for (int k = 0; k < NGE; ++k) {
        double um[NC], up[NC], fm[NC], fp[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          um[c] = hi[c][k];
          up[c] = s_x[xidx(c, k, line, pos + 1)];
        }
        point_flux<EQ>(um, dir, P, fm);
        point_flux<EQ>(up, dir, P, fp);
#pragma unroll
        for (int c = 0; c < NC; ++c) Fh[c][k] = 0.5 * (fm[c] + fp[c]) - 0.5 * alpha * (up[c] - um[c]);
      }
      double F0[NC][NGE];
      const bool do0 = ring_thread && ring_low;
      if (do0) {
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          double um[NC], up[NC], fm[NC], fp[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            um[c] = s_x0[(c * NGE + k) * TY + rpos];
            up[c] = s_x[xidx(c, k, rpos, 0)];
          }
          point_flux<EQ>(um, dir, P, fm);
          point_flux<EQ>(up, dir, P, fp);
#pragma unroll
          for (int c = 0; c < NC; ++c) F0[c][k] = 0.5 * (fm[c] + fp[c]) - 0.5 * alpha * (up[c] - um[c]);
        }
      }
      __syncthreads();
      // fluxes overwrite the traces: face pos + 1 by this cell, face 0 by the low ring
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) s_x[xidx(c, k, line, pos + 1)] = Fh[c][k];
      if (do0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int k = 0; k < NGE; ++k) s_x[xidx(c, k, rpos, 0)] = F0[c][k];
      }
    }
    __syncthreads();
    const double inv = 1.0 / (dir == 0 ? P.dx : P.dy);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double sdiff = 0.0, ssum = 0.0, smom = 0.0;
#pragma unroll
      for (int k = 0; k < NGE; ++k) {
        const double FL = s_x[xidx(c, k, line, pos)], FR = s_x[xidx(c, k, line, pos + 1)];
        sdiff = fma(wt[k], FR - FL, sdiff);
        ssum = fma(wt[k], FL + FR, ssum);
        smom = fma(wt[k] * node[k], FR - FL, smom);
      }
      RU[c] -= sdiff * inv;
      if (dir == 0) {
        RV[c] -= 0.5 * ssum * inv;
        RW[c] -= smom * inv;
      } else {
        RV[c] -= smom * inv;
        RW[c] -= 0.5 * ssum * inv;
      }
    }
    __syncthreads();   // the exchange buffer is reused by the next direction
  }

  // ---------------------------------------------------------------- epilogue
  const uint8_t myT = s_T[ly * LX + lx];
  double sp0 = 0.0, sp1 = 0.0;
  if (active) {
    const size_t gi = (size_t)gy * nx + gx;
    if (P.flagsT) P.flagsT[gi] = myT;
    if (P.flagsH) P.flagsH[gi] = hyb ? 1 : 0;
    double own[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) own[f] = S(s_in, f, ly, lx);   // limited stage input
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
        P.Tn[gi] = myT;
        if (myT) {
#pragma unroll
          for (int f = NC; f < NF; ++f) P.limn[(size_t)(f - NC) * plane + gi] = own[f];
        }
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
#define HW_L2(E, G) hipLaunchKernelGGL((hw::stage2d_kernel<E, G>), grid, block, 0, s, *P)
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

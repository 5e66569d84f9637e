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
#include "hw_device.h"
#include "hw_coeffs2d.h"

namespace hw {

constexpr int TX = 16, TY = 16, HL = 3, LX = TX + 2 * HL, LY = TY + 2 * HL, NT = TX * TY;
constexpr int NPOS = LX * LY;
constexpr int NXCD = 8;    // accelerator complex dies per MI355X
// hybrid cells per HWENO round (bounded so that two workgroups fit a CU's LDS)
template <int NGE>
constexpr int hw_round() { return NGE == 2 ? 128 : 32; }

template <int NGE>
struct Gauss;
template <>
struct Gauss<2> {
  static constexpr double node[2] = {-0.28867513459481288225457439025097873, 0.28867513459481288225457439025097873};
  static constexpr double wt[2] = {0.5, 0.5};
};
template <>
struct Gauss<3> {
  static constexpr double node[3] = {-0.38729833462074168851792653997823996, 0.0, 0.38729833462074168851792653997823996};
  static constexpr double wt[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};
};
// interior 3-point Gauss rule (volume integrals of eq. ode2)
__device__ constexpr double VW[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};

template <int NGE>
__device__ __forceinline__ void lin_edges(const double* in, int dir, double* lo, double* hi) {
  if constexpr (NGE == 2) {
    if (dir == 0) hw2::lin2d_xedges_ng2(in, lo, hi);
    else hw2::lin2d_yedges_ng2(in, lo, hi);
  } else {
    if (dir == 0) hw2::lin2d_xedges_ng3(in, lo, hi);
    else hw2::lin2d_yedges_ng3(in, lo, hi);
  }
}

template <int NGE>
__device__ __forceinline__ double edge_quartic(const double* c, int i) {
  if constexpr (NGE == 2) return hw2::edge_quartic_ng2(c, i);
  else return hw2::edge_quartic_ng3(c, i);
}
template <int NGE>
__device__ __forceinline__ double edge_quad(const double* c, int i) {
  if constexpr (NGE == 2) return hw2::edge_quad_ng2(c, i);
  else return hw2::edge_quad_ng3(c, i);
}

template <int n>
__device__ __forceinline__ void pq_coeffs(const double* w19, double* c) {
  if constexpr (n == 1) hw2::p1_coeffs(w19, c);
  else if constexpr (n == 2) hw2::p2_coeffs(w19, c);
  else if constexpr (n == 3) hw2::p3_coeffs(w19, c);
  else hw2::p4_coeffs(w19, c);
}

// Step 5.1 for one (characteristic) field: values at the edge points of direction dir
// (0: left then right points, 1: bottom then top points).  The combination
//   omega_0 (p0/gamma_0 - sum gamma_n/gamma_0 p_n) + sum omega_n p_n
// is accumulated as sum a_n p_n with a_0 = omega_0/gamma_0, a_n = omega_n - omega_0
// gamma_n/gamma_0, so each candidate's coefficients are built, used and dropped in turn.
template <int NGE, int n>
__device__ __forceinline__ void hweno_beta(const double* w19, double* beta) {
  double c[6];
  pq_coeffs<n>(w19, c);
  beta[n] = hw2::beta_pq(c);
}
template <int NGE, int n>
__device__ __forceinline__ void hweno_add(const double* w19, double an, int dir, double* vals) {
  double c[6];
  pq_coeffs<n>(w19, c);
#pragma unroll
  for (int k = 0; k < 2 * NGE; ++k) vals[k] = fma(an, edge_quad<NGE>(c, dir * 2 * NGE + k), vals[k]);
}

template <int NGE>
__device__ __forceinline__ void hweno2d_field(const double* w19, const Weights& W, int dir,
                                              double* vals /* 2*NGE */) {
  double beta[5], om[5];
  {
    double c[15];
    hw2::p0_coeffs(w19, c);
    beta[0] = hw2::beta_p0(c);
  }
  hweno_beta<NGE, 1>(w19, beta);
  hweno_beta<NGE, 2>(w19, beta);
  hweno_beta<NGE, 3>(w19, beta);
  hweno_beta<NGE, 4>(w19, beta);
  nonlinear_weights<4>(beta, W.rec, W.eps, om);
  {
    const double a0 = om[0] / W.rec[0];
    double c[15];
    hw2::p0_coeffs(w19, c);
#pragma unroll
    for (int k = 0; k < 2 * NGE; ++k) vals[k] = a0 * edge_quartic<NGE>(c, dir * 2 * NGE + k);
  }
  hweno_add<NGE, 1>(w19, om[1] - om[0] * (W.rec[1] / W.rec[0]), dir, vals);
  hweno_add<NGE, 2>(w19, om[2] - om[0] * (W.rec[2] / W.rec[0]), dir, vals);
  hweno_add<NGE, 3>(w19, om[3] - om[0] * (W.rec[3] / W.rec[0]), dir, vals);
  hweno_add<NGE, 4>(w19, om[4] - om[0] * (W.rec[4] / W.rec[0]), dir, vals);
}

__device__ __forceinline__ double S(const double* s, int f, int ly, int lx) {
  return s[(f * LY + ly) * LX + lx];
}

// the 19 stencil values of field component c (moment-major fields) around (ly, lx)
template <int NC>
__device__ __forceinline__ void gather19(const double* s, int c, int ly, int lx, double* in) {
#pragma unroll
  for (int k = 0; k < 9; ++k) in[k] = S(s, c, ly + k / 3 - 1, lx + k % 3 - 1);
  const int cy[5] = {-1, 0, 0, 0, 1}, cx[5] = {0, -1, 0, 1, 0};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    in[9 + k] = S(s, NC + c, ly + cy[k], lx + cx[k]);
    in[14 + k] = S(s, 2 * NC + c, ly + cy[k], lx + cx[k]);
  }
}

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
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous raster
  // range of tiles so that neighbouring tiles (whose halos overlap) share its L2.
  int bx, by;
  {
    const int ntx = (nx + TX - 1) / TX;
    const int N = gridDim.x, id = blockIdx.x;
    const int xcd = id % NXCD, k = id / NXCD;
    const int per = N / NXCD, rem = N % NXCD;
    const int t = xcd * per + (xcd < rem ? xcd : rem) + k;
    by = t / ntx;
    bx = t - by * ntx;
  }
  const int gx0 = bx * TX - HL, gy0 = by * TY - HL;
  const size_t plane = (size_t)nx * ny;

  // ---------------------------------------------------------------- stage input -> LDS
  for (int p = tid; p < NPOS; p += NT) {
    const int ly = p / LX, lx = p - ly * LX;
    double sx, sy;
    const int gx = map_index(gx0 + lx, nx, P.bcx, sx);
    const int gy = map_index(gy0 + ly, ny, P.bcy, sy);
    const double* src = P.in + (size_t)gy * nx + gx;
    double v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = src[f * plane];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int m = f / NC;
      s_in[f * NPOS + p] = m == 1 ? sx * v[f] : (m == 2 ? sy * v[f] : v[f]);
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- flags on tile+2
  constexpr int R2 = LX - 2;   // 20
  for (int q = tid; q < R2 * R2; q += NT) {
    const int ly = 1 + q / R2, lx = 1 + q % R2;
    uint8_t t = 0;
    if (P.tc_mode == TC_ALL) {
      t = 1;
    } else if (P.tc_mode == TC_KXRCF) {
      double velx, vely;
      if constexpr (EQ == EQ_EULER) {
        const double rho = S(s_in, 0, ly, lx);
        velx = S(s_in, 1, ly, lx) / rho;
        vely = S(s_in, 2, ly, lx) / rho;
      } else if constexpr (EQ == EQ_BURGERS) {
        velx = vely = S(s_in, 0, ly, lx);
      } else {
        velx = P.adv0;
        vely = P.adv1;
      }
      constexpr int ncheck = (EQ == EQ_EULER) ? 2 : 1;
#pragma unroll
      for (int k = 0; k < ncheck; ++k) {
        const int c = (k == 0) ? 0 : NC - 1;   // density, then energy
        double cc[3], l[3], r[3], b[3], tt[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          cc[m] = S(s_in, m * NC + c, ly, lx);
          l[m] = S(s_in, m * NC + c, ly, lx - 1);
          r[m] = S(s_in, m * NC + c, ly, lx + 1);
          b[m] = S(s_in, m * NC + c, ly - 1, lx);
          tt[m] = S(s_in, m * NC + c, ly + 1, lx);
        }
        if (kxrcf2d(cc, l, r, b, tt, velx, vely, P.dx, P.dy, P.h)) t = 1;
      }
    }
    s_T[ly * LX + lx] = t;
  }
  __syncthreads();

  // ---------------------------------------------------------------- limiter (Jacobi)
  if (P.tc_mode != TC_NONE) {
    double limv[2][2 * NC];
    bool limdo[2] = {false, false};
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int q = tid + rep * NT;
      if (q >= R2 * R2) break;
      const int ly = 1 + q / R2, lx = 1 + q % R2;
      if (!s_T[ly * LX + lx]) continue;
      limdo[rep] = true;
      if constexpr (EQ != EQ_EULER) {
        limv[rep][0] = limit_moment(S(s_in, 0, ly, lx - 1), S(s_in, 0, ly, lx),
                                    S(s_in, 0, ly, lx + 1), S(s_in, 1, ly, lx - 1),
                                    S(s_in, 1, ly, lx + 1), P.w.lim, P.w.eps);
        limv[rep][1] = limit_moment(S(s_in, 0, ly - 1, lx), S(s_in, 0, ly, lx),
                                    S(s_in, 0, ly + 1, lx), S(s_in, 2, ly - 1, lx),
                                    S(s_in, 2, ly + 1, lx), P.w.lim, P.w.eps);
      } else {
        double U[4];
        for (int c = 0; c < 4; ++c) U[c] = S(s_in, c, ly, lx);
        for (int dir = 0; dir < 2; ++dir) {
          const int oy = dir, ox = 1 - dir;   // neighbour offsets along the line
          const int mf = 1 + dir;             // moment being limited
          double out[4] = {0.0, 0.0, 0.0, 0.0};
          for (int f = 0; f < 4; ++f) {
            double Lr[4], Rc[4];
            euler_eig2d_field(U, P.gam, dir, f, Lr, Rc);
            double um = 0.0, u0 = 0.0, up = 0.0, vm = 0.0, vp = 0.0;
            for (int c = 0; c < 4; ++c) {
              const double l = Lr[c];
              um = fma(l, S(s_in, c, ly - oy, lx - ox), um);
              u0 = fma(l, S(s_in, c, ly, lx), u0);
              up = fma(l, S(s_in, c, ly + oy, lx + ox), up);
              vm = fma(l, S(s_in, mf * 4 + c, ly - oy, lx - ox), vm);
              vp = fma(l, S(s_in, mf * 4 + c, ly + oy, lx + ox), vp);
            }
            const double vc = limit_moment(um, u0, up, vm, vp, P.w.lim, P.w.eps);
            for (int c = 0; c < 4; ++c) out[c] = fma(Rc[c], vc, out[c]);
          }
          for (int c = 0; c < 4; ++c) limv[rep][dir * 4 + c] = out[c];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      if (!limdo[rep]) continue;
      const int q = tid + rep * NT;
      const int ly = 1 + q / R2, lx = 1 + q % R2;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        s_in[((NC + c) * LY + ly) * LX + lx] = limv[rep][c];
        s_in[((2 * NC + c) * LY + ly) * LX + lx] = limv[rep][NC + c];
      }
    }
  }
  // ---------------------------------------------------------------- hybrid mask, tile+1
  constexpr int R1 = LX - 4;   // 18
  for (int q = tid; q < R1 * R1; q += NT) {
    const int ly = 2 + q / R1, lx = 2 + q % R1;
    uint8_t hm = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) hm |= s_T[(ly + dy) * LX + lx + dx];
    s_H[ly * LX + lx] = hm;
  }
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

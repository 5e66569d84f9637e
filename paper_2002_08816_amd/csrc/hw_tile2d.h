// Tile geometry and the phases shared by the two-dimensional stage kernel and its adjoint
// (Zhao & Qiu, arXiv 2002.08816, Section 2.2): staging of a tile plus ghost layers in LDS,
// KXRCF flags (Step 4, Remark 3), the Jacobi limiter of the first moments (Step 4,
// Remark 4), the hybrid mask, and the per-cell reconstructions of Steps 5.1-5.2.
// The adjoint re-derives flags, limited moments and hybrid masks of a stored stage input
// through these same functions, so they agree bit for bit with the forward stage.
#pragma once
#include "hw_device.h"
#include "hw_coeffs2d.h"

namespace hw {

constexpr int TX = 16, TY = 16, HL = 3, LX = TX + 2 * HL, LY = TY + 2 * HL, NT = TX * TY;
constexpr int NPOS = LX * LY;
constexpr int NXCD = 8;    // accelerator complex dies per MI355X
constexpr int R2 = LX - 2;   // tile+2 (flags, limiter)
constexpr int R1 = LX - 4;   // tile+1 (hybrid mask, ring cells)

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

// smoothness indicators of the five candidates and the nonlinear weights (eq. tao4)
template <int NGE>
__device__ __forceinline__ void hweno2d_weights(const double* w19, const Weights& W, double* beta,
                                                double* om) {
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
}

// the combination of Step 5.1 with given nonlinear weights
template <int NGE>
__device__ __forceinline__ void hweno2d_combine(const double* w19, const Weights& W, int dir,
                                                const double* om, double* vals /* 2*NGE */) {
  const double ig0 = rcp_nr(W.rec[0]);
  {
    const double a0 = om[0] * ig0;
    double c[15];
    hw2::p0_coeffs(w19, c);
#pragma unroll
    for (int k = 0; k < 2 * NGE; ++k) vals[k] = a0 * edge_quartic<NGE>(c, dir * 2 * NGE + k);
  }
  hweno_add<NGE, 1>(w19, om[1] - om[0] * (W.rec[1] * ig0), dir, vals);
  hweno_add<NGE, 2>(w19, om[2] - om[0] * (W.rec[2] * ig0), dir, vals);
  hweno_add<NGE, 3>(w19, om[3] - om[0] * (W.rec[3] * ig0), dir, vals);
  hweno_add<NGE, 4>(w19, om[4] - om[0] * (W.rec[4] * ig0), dir, vals);
}

template <int NGE>
__device__ __forceinline__ void hweno2d_field(const double* w19, const Weights& W, int dir,
                                              double* vals /* 2*NGE */) {
  double beta[5], om[5];
  hweno2d_weights<NGE>(w19, W, beta, om);
  hweno2d_combine<NGE>(w19, W, dir, om, vals);
}

// LDS tile of W x W positions per field (W = LX: three ghost layers)
template <int W = LX>
__device__ __forceinline__ double S(const double* s, int f, int ly, int lx) {
  return s[(f * W + ly) * W + lx];
}

// the 19 stencil values of field component c (moment-major fields) around (ly, lx)
template <int NC, int W = LX>
__device__ __forceinline__ void gather19(const double* s, int c, int ly, int lx, double* in) {
#pragma unroll
  for (int k = 0; k < 9; ++k) in[k] = S<W>(s, c, ly + k / 3 - 1, lx + k % 3 - 1);
  const int cy[5] = {-1, 0, 0, 0, 1}, cx[5] = {0, -1, 0, 1, 0};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    in[9 + k] = S<W>(s, NC + c, ly + cy[k], lx + cx[k]);
    in[14 + k] = S<W>(s, 2 * NC + c, ly + cy[k], lx + cx[k]);
  }
}


// Tile (bx, by) of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin; each
// XCD gets a contiguous raster range of tiles so that neighbouring tiles (whose halos
// overlap) share its L2.
__device__ __forceinline__ void tile_of_block(int nx, int& bx, int& by) {
  const int ntx = (nx + TX - 1) / TX;
  const int N = gridDim.x, id = blockIdx.x;
  const int xcd = id % NXCD, k = id / NXCD;
  const int per = N / NXCD, rem = N % NXCD;
  const int t = xcd * per + (xcd < rem ? xcd : rem) + k;
  by = t / ntx;
  bx = t - by * ntx;
}

// KXRCF flags (Step 4; Euler: density or energy fires) on the positions [lo, LX - lo)^2
// (lo = 1: tile+2, reading tile+3)
template <int EQ>
__device__ __forceinline__ void flags_tile(const double* s_in, int tc_mode, double adv0, double adv1,
                                           double dx, double dy, double h, uint8_t* s_T,
                                           int lo = 1) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  const int w = LX - 2 * lo;
  for (int q = threadIdx.x; q < w * w; q += NT) {
    const int ly = lo + q / w, lx = lo + q % w;
    uint8_t t = 0;
    if (tc_mode == TC_ALL) {
      t = 1;
    } else if (tc_mode == TC_KXRCF) {
      double velx, vely;
      if constexpr (EQ == EQ_EULER) {
        const double rho = S(s_in, 0, ly, lx);
        velx = S(s_in, 1, ly, lx) / rho;
        vely = S(s_in, 2, ly, lx) / rho;
      } else if constexpr (EQ == EQ_BURGERS) {
        velx = vely = S(s_in, 0, ly, lx);
      } else {
        velx = adv0;
        vely = adv1;
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
        if (kxrcf2d(cc, l, r, b, tt, velx, vely, dx, dy, h)) t = 1;
      }
    }
    s_T[ly * LX + lx] = t;
  }
}

// Limiter of the first moments on the flagged cells of [lo, LX - lo)^2 (lo = 1: tile+2),
// dimension by dimension, characteristic-wise for Euler; Jacobi: every value from the
// unmodified input, written back after a barrier.  Call only when tc_mode != TC_NONE (it
// synchronises the block).
template <int EQ>
__device__ __forceinline__ void limit_tile(double* s_in, const uint8_t* s_T, double gam,
                                           const Weights& w, int lo = 1) {
  constexpr int NC = (EQ == EQ_EULER) ? 4 : 1;
  const int tid = threadIdx.x;
  const int rw = LX - 2 * lo;
  double limv[2][2 * NC];
  bool limdo[2] = {false, false};
#pragma unroll
  for (int rep = 0; rep < 2; ++rep) {
    const int q = tid + rep * NT;
    if (q >= rw * rw) break;
    const int ly = lo + q / rw, lx = lo + q % rw;
    if (!s_T[ly * LX + lx]) continue;
    limdo[rep] = true;
    if constexpr (EQ != EQ_EULER) {
      limv[rep][0] = limit_moment(S(s_in, 0, ly, lx - 1), S(s_in, 0, ly, lx),
                                  S(s_in, 0, ly, lx + 1), S(s_in, 1, ly, lx - 1),
                                  S(s_in, 1, ly, lx + 1), w.lim, w.eps);
      limv[rep][1] = limit_moment(S(s_in, 0, ly - 1, lx), S(s_in, 0, ly, lx),
                                  S(s_in, 0, ly + 1, lx), S(s_in, 2, ly - 1, lx),
                                  S(s_in, 2, ly + 1, lx), w.lim, w.eps);
    } else {
      double U[4];
      for (int c = 0; c < 4; ++c) U[c] = S(s_in, c, ly, lx);
      for (int dir = 0; dir < 2; ++dir) {
        const int oy = dir, ox = 1 - dir;   // neighbour offsets along the line
        const int mf = 1 + dir;             // moment being limited
        double out[4] = {0.0, 0.0, 0.0, 0.0};
        for (int f = 0; f < 4; ++f) {
          double Lr[4], Rc[4];
          euler_eig2d_field(U, gam, dir, f, Lr, Rc);
          double um = 0.0, u0 = 0.0, up = 0.0, vm = 0.0, vp = 0.0;
          for (int c = 0; c < 4; ++c) {
            const double l = Lr[c];
            um = fma(l, S(s_in, c, ly - oy, lx - ox), um);
            u0 = fma(l, S(s_in, c, ly, lx), u0);
            up = fma(l, S(s_in, c, ly + oy, lx + ox), up);
            vm = fma(l, S(s_in, mf * 4 + c, ly - oy, lx - ox), vm);
            vp = fma(l, S(s_in, mf * 4 + c, ly + oy, lx + ox), vp);
          }
          const double vc = limit_moment(um, u0, up, vm, vp, w.lim, w.eps);
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
    const int ly = lo + q / rw, lx = lo + q % rw;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      s_in[((NC + c) * LY + ly) * LX + lx] = limv[rep][c];
      s_in[((2 * NC + c) * LY + ly) * LX + lx] = limv[rep][NC + c];
    }
  }
}

// hybrid mask: a flag anywhere in the 3x3 block (Step 5), on [lo, LX - lo)^2 (lo = 2:
// tile+1)
__device__ __forceinline__ void hybrid_tile(const uint8_t* s_T, uint8_t* s_H, int lo = 2) {
  const int w = LX - 2 * lo;
  for (int q = threadIdx.x; q < w * w; q += NT) {
    const int ly = lo + q / w, lx = lo + q % w;
    uint8_t hm = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) hm |= s_T[(ly + dy) * LX + lx + dx];
    s_H[ly * LX + lx] = hm;
  }
}

}  // namespace hw

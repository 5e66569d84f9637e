// The one-dimensional stage on a mesh of cells of different sizes (Zhao & Qiu, arXiv
// 2002.08816, Section 2.1).  The scheme defines each polynomial by moment conditions on
// the cells of its stencil and combines them with artificial linear weights that do not
// depend on the geometry; on cells of different sizes only the polynomials change.  In
// the local coordinate xi = (x - x_i)/dx_i of cell I_i the neighbours are [-1/2 - a, -1/2]
// and [1/2, 1/2 + b] (a = dx_{i-1}/dx_i, b = dx_{i+1}/dx_i); the average of p over a cell
// of centre c and width w is (1/w) int p dxi, its first moment (1/w) int p (xi - c)/w dxi.
// A setup kernel solves these conditions once per cell and stores, per cell, every linear
// functional and smoothness-indicator factor the stage needs (a table of NTAB doubles,
// stored field by field); the stage kernel evaluates them instead of the printed
// uniform-mesh formulas.
//
// Smoothness indicators (eq. GHYZ on I_i in xi): beta = c^T G c for the monomial
// coefficients c of the polynomial, G = sum_l int D^l xi^m D^l xi^n; stored as the rows of
// R C with G = R^T R on the non-constant monomials, so that beta = sum_r (row_r . d)^2.
#pragma once
#include "hw_device.h"

namespace hw {
namespace mesh1d {

// table entries (stencil data d5 = (u_{-1}, u_0, u_{+1}, v_{-1}, v_{+1}) for the limiter,
// d6 = (u_{-1}, u_0, u_{+1}, v_{-1}, v_0, v_{+1}) for the reconstruction)
enum {
  K_DX = 0,
  K_LQ0 = 1,    // first moment over I_i of the Step-1 quartic: 5 (d5)
  K_LQ1 = 6,    // ... of the linear q1 on {I_{i-1}, I_i}: 2 (u_{-1}, u_0)
  K_LQ2 = 8,    // ... of the linear q2 on {I_i, I_{i+1}}: 2 (u_0, u_{+1})
  K_LB0 = 10,   // indicator rows of the quartic: 4 x 5
  K_LB1 = 30,   // slope of q1: 2
  K_LB2 = 32,   // slope of q2: 2
  K_RL0 = 34,   // Step-2 quintic at xi = -1/2: 6 (d6)
  K_RR0 = 40,   // ... at xi = +1/2
  K_RIM = 46,   // ... at xi = -sqrt5/10
  K_RIP = 52,   // ... at xi = +sqrt5/10
  K_RL1 = 58,   // quadratic p1 (u_{-1}, u_0, v_0) at -1/2: 3
  K_RR1 = 61,   // ... at +1/2
  K_RL2 = 64,   // quadratic p2 (u_0, u_{+1}, v_0) at -1/2: 3
  K_RR2 = 67,   // ... at +1/2
  K_RB0 = 70,   // indicator rows of the quintic: 5 x 6
  K_RB1 = 100,  // indicator rows of p1: 2 x 3
  K_RB2 = 106,  // indicator rows of p2: 2 x 3
  NTAB = 112
};

struct Tab {
  const double* t;
  size_t n;   // cells (the table's field stride)
  int i;      // cell
  __device__ __forceinline__ double operator[](int k) const { return t[(size_t)k * n + i]; }
};

template <int N>
__device__ __forceinline__ double dot(const Tab& T, int k, const double* d) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) s = fma(T[k + j], d[j], s);
  return s;
}

// Step 1: the modified first moment of the cell (limit_moment on this cell's geometry)
__device__ __forceinline__ double limit_moment_nu(const Tab& T, double um, double u0, double up,
                                                  double vm, double vp, const double* g, double eps) {
  const double d5[5] = {um, u0, up, vm, vp};
  const double d2m[2] = {um, u0}, d2p[2] = {u0, up};
  double q[3], b[3], om[3];
  q[0] = dot<5>(T, K_LQ0, d5);
  q[1] = dot<2>(T, K_LQ1, d2m);
  q[2] = dot<2>(T, K_LQ2, d2p);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double e = dot<5>(T, K_LB0 + 5 * r, d5);
    s = fma(e, e, s);
  }
  b[0] = s;
  const double s1 = dot<2>(T, K_LB1, d2m), s2 = dot<2>(T, K_LB2, d2p);
  b[1] = s1 * s1;
  b[2] = s2 * s2;
  nonlinear_weights<2>(b, g, eps, om);
  return weno_combine<2>(om, g, q);
}

// Step 2.2 / 2.3: the quintic at the faces and the interior Gauss-Lobatto points
__device__ __forceinline__ void linear1d_nu(const Tab& T, const double* d6, double& left,
                                            double& right, double& im, double& ip) {
  left = dot<6>(T, K_RL0, d6);
  right = dot<6>(T, K_RR0, d6);
  im = dot<6>(T, K_RIM, d6);
  ip = dot<6>(T, K_RIP, d6);
}

// Step 2.1: HWENO values at both faces (one set of nonlinear weights)
__device__ __forceinline__ void hweno1d_nu(const Tab& T, const double* d6, const double* g,
                                           double eps, double& left, double& right) {
  const double d1[3] = {d6[0], d6[1], d6[4]}, d2[3] = {d6[1], d6[2], d6[4]};
  double ql[3], qr[3], b[3], om[3];
  ql[0] = dot<6>(T, K_RL0, d6);
  qr[0] = dot<6>(T, K_RR0, d6);
  ql[1] = dot<3>(T, K_RL1, d1);
  qr[1] = dot<3>(T, K_RR1, d1);
  ql[2] = dot<3>(T, K_RL2, d2);
  qr[2] = dot<3>(T, K_RR2, d2);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const double e = dot<6>(T, K_RB0 + 6 * r, d6);
    s = fma(e, e, s);
  }
  b[0] = s;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double e1 = dot<3>(T, K_RB1 + 3 * r, d1), e2 = dot<3>(T, K_RB2 + 3 * r, d2);
    s1 = fma(e1, e1, s1);
    s2 = fma(e2, e2, s2);
  }
  b[1] = s1;
  b[2] = s2;
  nonlinear_weights<2>(b, g, eps, om);
  left = weno_combine<2>(om, g, ql);
  right = weno_combine<2>(om, g, qr);
}

}  // namespace mesh1d
}  // namespace hw

// Per-cell tables of every instance of a batch on cells of different sizes (stage1d.hip):
// faces (device) holds instance b's n_b + 1 face coordinates after those of the instances
// before it; off (host) the instance offsets [ninst + 1]; tab the [NTAB][total] tables.
extern "C" hipError_t hw_launch_mesh1d_setup_batch(const double* faces, const int* off, int ninst,
                                                   int bc, double* tab, int total, hipStream_t s);

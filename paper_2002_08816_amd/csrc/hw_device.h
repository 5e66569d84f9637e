// Device-side building blocks of the hybrid Hermite WENO stage operator
// (Zhao & Qiu, arXiv 2002.08816): fluxes, characteristic fields, the Step-1 limiter,
// the Step-2 one-dimensional reconstructions, the KXRCF indicator and reductions.
// All arithmetic is FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hw_stage.h"

namespace hw {

// 1/x from the hardware reciprocal estimate and two Newton steps, within one ulp of the
// rounded quotient.  Used where a quotient feeds continuous arithmetic (fluxes,
// eigenvectors, nonlinear weights); never where a comparison decides a flag.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// stage coefficients (a, b): out = a * W(u^n) + b * (W(u^(s)) + dt L(W(u^(s))))
__device__ __forceinline__ void rk_coeffs(int mode, double& a, double& b) {
  if (mode == MODE_RK2) { a = 0.75; b = 0.25; }
  else if (mode == MODE_RK3) { a = 1.0 / 3.0; b = 2.0 / 3.0; }
  else { a = 0.0; b = 1.0; }
}

// ------------------------------------------------------------------ boundary mapping
// Maps a global cell index (possibly a ghost) to a stored index.  Returns the sign that
// the first moment normal to this boundary picks up (transmissive and reflective: the
// mirror; a reflective wall also negates the normal momentum, which its caller applies).
__device__ __forceinline__ int map_index(int g, int n, int bc, double& sgn) {
  sgn = 1.0;
  if (bc == BC_PERIODIC) {
    if (g < 0) g += n;
    else if (g >= n) g -= n;
    if (g < 0 || g >= n) {   // only for meshes narrower than a tile plus its halo
      g %= n;
      if (g < 0) g += n;
    }
    return g;
  }
  if (g < 0) { g = -g - 1; sgn = -1.0; }
  else if (g >= n) { g = 2 * n - 1 - g; sgn = -1.0; }
  // cells further out than the ghost layers are never used by an active cell; clamp
  if (g < 0) g = 0;
  if (g >= n) g = n - 1;
  return g;
}

// ------------------------------------------------------------------ atomics / reductions
__device__ __forceinline__ void atomic_max_pos(unsigned long long* addr, double v) {
  // v >= 0: the IEEE bit pattern orders like the value, so an integer max is exact
  if (!(v >= 0.0)) v = __longlong_as_double(0x7ff0000000000000ull);   // NaN -> +inf
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// Speeds of both directions from their ASPREAD partial maxima (non-negative doubles, so the
// largest bit pattern is the largest value); call with the whole first wave, result in
// out[0..1] of LDS after a barrier.
__device__ __forceinline__ void reduce_speeds(const unsigned long long* a, double* out) {
  if (threadIdx.x < 64) {
    unsigned long long m0 = 0ull, m1 = 0ull;
    if (threadIdx.x < ASPREAD) {
      m0 = a[threadIdx.x];
      m1 = a[ASPREAD + threadIdx.x];
    }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long x0 = __shfl_xor(m0, o, 64), x1 = __shfl_xor(m1, o, 64);
      m0 = x0 > m0 ? x0 : m0;
      m1 = x1 > m1 ? x1 : m1;
    }
    if (threadIdx.x == 0) {
      out[0] = __longlong_as_double((long long)m0);
      out[1] = __longlong_as_double((long long)m1);
    }
  }
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// block-wide max over 256 threads (4 waves); red must hold 4 doubles
__device__ __forceinline__ double block_max256(double v, double* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ------------------------------------------------------------------ nonlinear weights
// eqs. tao5 / tao4 and the weights below them: tau = (mean |beta_0 - beta_n|)^2,
// wbar_n = gamma_n (1 + tau / (beta_n + eps)), omega = wbar / sum(wbar).
template <int K>
__device__ __forceinline__ void nonlinear_weights(const double* beta, const double* g, double eps,
                                                  double* om) {
  double s = 0.0;
#pragma unroll
  for (int n = 1; n <= K; ++n) s += fabs(beta[0] - beta[n]);
  s = s / (double)K;
  const double tau = s * s;
  double tot = 0.0;
#pragma unroll
  for (int n = 0; n <= K; ++n) {
    om[n] = g[n] * (1.0 + tau * rcp_nr(beta[n] + eps));
    tot += om[n];
  }
  const double it = rcp_nr(tot);
#pragma unroll
  for (int n = 0; n <= K; ++n) om[n] = om[n] * it;
}

// value = omega_0 (q_0/gamma_0 - sum gamma_n/gamma_0 q_n) + sum omega_n q_n   (eq. p_big)
template <int K>
__device__ __forceinline__ double weno_combine(const double* om, const double* g, const double* q) {
  const double ig0 = rcp_nr(g[0]);
  double lin = q[0] * ig0;
#pragma unroll
  for (int n = 1; n <= K; ++n) lin -= g[n] * ig0 * q[n];
  double v = om[0] * lin;
#pragma unroll
  for (int n = 1; n <= K; ++n) v += om[n] * q[n];
  return v;
}

// ------------------------------------------------------------------ Step 1 limiter
// Modified first moment of I_i from the averages of I_{i-1}, I_i, I_{i+1} and the first
// moments of I_{i-1}, I_{i+1} (Section 2.1 Step 1; the smoothness indicator of the
// quartic is the definition eq. GHYZ with r = 4, i.e. the printed form with the first
// moments entering its last square with factor 6).
__device__ __forceinline__ void limiter_terms(double um, double u0, double up, double vm, double vp,
                                              double* q, double* t, double* b) {
  q[0] = (5.0 / 76.0) * (up - um) - (11.0 / 38.0) * (vm + vp);
  q[1] = (u0 - um) * (1.0 / 12.0);
  q[2] = (up - u0) * (1.0 / 12.0);
  t[0] = (29.0 / 38.0) * (um - up) + (60.0 / 19.0) * (vm + vp);
  t[1] = (9.0 / 4.0) * (um + up) - (9.0 / 2.0) * u0 + (15.0 / 2.0) * (vm - vp);
  t[2] = (um - up) + 12.0 * (vm + vp);
  t[3] = (5.0 / 2.0) * (um + up) - 5.0 * u0 + 9.0 * (vm - vp);
  t[4] = (um - 2.0 * u0 + up) + 6.0 * (vm - vp);
  b[0] = t[0] * t[0] + t[1] * t[1] + (3905.0 / 1444.0) * (t[2] * t[2]) + (1.0 / 12.0) * (t[3] * t[3]) +
         (109341.0 / 448.0) * (t[4] * t[4]);
  b[1] = (u0 - um) * (u0 - um);
  b[2] = (up - u0) * (up - u0);
}

__device__ __forceinline__ double limit_moment(double um, double u0, double up, double vm, double vp,
                                               const double* g, double eps) {
  double q[3], t[5], b[3], om[3];
  limiter_terms(um, u0, up, vm, vp, q, t, b);
  nonlinear_weights<2>(b, g, eps, om);
  return weno_combine<2>(om, g, q);
}

// ------------------------------------------------------------------ Step 2 (1D)
// Linear interface values u^+_{i-1/2}, u^-_{i+1/2} (Step 2.2) and interior values
// u_{i -/+ sqrt5/10} (Step 2.3), written through their mirror-even and mirror-odd parts.
__device__ __forceinline__ void linear1d(double um, double u0, double up, double vm, double v0,
                                         double vp, double& left, double& right, double& im,
                                         double& ip) {
  const double su = um + up, du = up - um, sv = vm + vp, dv = vm - vp;
  const double E = (7.0 / 12.0) * u0 + (5.0 / 24.0) * su + 0.75 * dv;
  const double O = (19.0 / 216.0) * du - (31.0 / 108.0) * sv + (241.0 / 54.0) * v0;
  left = E - O;
  right = E + O;
  const double s5 = 2.23606797749978969640917366873127624;  // sqrt(5)
  const double Ei = (13.0 / 12.0) * u0 - (1.0 / 24.0) * su - 0.15 * dv;
  const double Oi = s5 * ((-101.0 / 5400.0) * du + (841.0 / 13500.0) * sv + (10289.0 / 6750.0) * v0);
  im = Ei - Oi;
  ip = Ei + Oi;
}

// HWENO interface values (Step 2.1): quintic p0 and quadratics p1, p2 at x_{i+1/2} as
// printed; at x_{i-1/2} their mirror images.  One set of nonlinear weights serves both
// faces.
__device__ __forceinline__ void hweno1d(double um, double u0, double up, double vm, double v0,
                                        double vp, const double* g, double eps, double& left,
                                        double& right) {
  double b[3], om[3], qr[3], ql[3];
  qr[0] = (13.0 / 108.0) * um + (7.0 / 12.0) * u0 + (8.0 / 27.0) * up + (25.0 / 54.0) * vm +
          (241.0 / 54.0) * v0 - (28.0 / 27.0) * vp;
  ql[0] = (8.0 / 27.0) * um + (7.0 / 12.0) * u0 + (13.0 / 108.0) * up + (28.0 / 27.0) * vm -
          (241.0 / 54.0) * v0 - (25.0 / 54.0) * vp;
  qr[1] = (1.0 / 6.0) * um + (5.0 / 6.0) * u0 + 8.0 * v0;
  ql[1] = (1.0 / 6.0) * um + (5.0 / 6.0) * u0 - 4.0 * v0;
  qr[2] = (5.0 / 6.0) * u0 + (1.0 / 6.0) * up + 4.0 * v0;
  ql[2] = (5.0 / 6.0) * u0 + (1.0 / 6.0) * up - 8.0 * v0;
  const double a1 = (19.0 / 108.0) * (um - up) + (31.0 / 54.0) * (vm + vp) - (241.0 / 27.0) * v0;
  const double a2 = (9.0 / 4.0) * (um + up) - (9.0 / 2.0) * u0 + (15.0 / 2.0) * (vm - vp);
  const double a3 = (70.0 / 9.0) * (um - up) + (200.0 / 9.0) * (vm + vp) + (1280.0 / 9.0) * v0;
  const double a4 = (5.0 / 2.0) * (um + up) - 5.0 * u0 + 9.0 * (vm - vp);
  const double a5 = (175.0 / 18.0) * (um - up) + (277.0 / 9.0) * (vm + vp) + (1546.0 / 9.0) * v0;
  const double a6 = (95.0 / 18.0) * (um - up) + (155.0 / 9.0) * (vm + vp) + (830.0 / 9.0) * v0;
  const double a7 = (5.0 / 8.0) * (um + up) - (5.0 / 4.0) * u0 + (15.0 / 4.0) * (vm - vp);
  const double a8 = (35.0 / 36.0) * (um - up) + (77.0 / 18.0) * (vm + vp) + (133.0 / 9.0) * v0;
  b[0] = a1 * a1 + a2 * a2 + a3 * a3 + (1.0 / 12.0) * (a4 * a4) + (1.0 / 12.0) * (a5 * a5) +
         (1.0 / 180.0) * (a6 * a6) + (109341.0 / 175.0) * (a7 * a7) +
         (27553933.0 / 1764.0) * (a8 * a8);
  const double c1 = um - u0 + 12.0 * v0, c2 = u0 - up + 12.0 * v0;
  b[1] = 144.0 * v0 * v0 + (13.0 / 3.0) * (c1 * c1);
  b[2] = 144.0 * v0 * v0 + (13.0 / 3.0) * (c2 * c2);
  nonlinear_weights<2>(b, g, eps, om);
  left = weno_combine<2>(om, g, ql);
  right = weno_combine<2>(om, g, qr);
}

// ------------------------------------------------------------------ KXRCF indicator
// Reading of the indicator of Krivodonova et al. on the P1 polynomial of the moments:
// mean traces ubar -/+ 6 vbar (left/right) and ubar -/+ 6 wbar (bottom/top), inflow
// faces from the velocity at the cell average, troubled iff
//   |sum_inflow |e| (trace_K - trace_nb)| > h |dK^-| (|ubar| + 6|vbar| + 6|wbar|).
// Evaluated without contraction so that the same inputs give the same decision as a
// plain evaluation in the stated order.
__device__ __forceinline__ bool kxrcf1d(double ub, double vb, double ubl, double vbl, double ubr,
                                        double vbr, double vel, double h) {
#pragma clang fp contract(off)
  const bool lin = vel > 0.0, rin = vel < 0.0;
  if (!lin && !rin) return false;
  const double jl = (ub - 6.0 * vb) - (ubl + 6.0 * vbl);
  const double jr = (ub + 6.0 * vb) - (ubr - 6.0 * vbr);
  const double s = (lin ? jl : 0.0) + (rin ? jr : 0.0);
  const double len = (lin ? 1.0 : 0.0) + (rin ? 1.0 : 0.0);
  const double nrm = fabs(ub) + 6.0 * fabs(vb);
  return fabs(s) > h * len * nrm;
}

// (inflow faces given: lin = velx > 0, rin = velx < 0, bin = vely > 0, tin = vely < 0)
__device__ __forceinline__ bool kxrcf2d_in(const double* c, const double* l, const double* r,
                                           const double* b, const double* t, bool lin, bool rin,
                                           bool bin, bool tin, double dx, double dy, double h) {
#pragma clang fp contract(off)
  if (!(lin || rin || bin || tin)) return false;
  const double jl = (c[0] - 6.0 * c[1]) - (l[0] + 6.0 * l[1]);
  const double jr = (c[0] + 6.0 * c[1]) - (r[0] - 6.0 * r[1]);
  const double jb = (c[0] - 6.0 * c[2]) - (b[0] + 6.0 * b[2]);
  const double jt = (c[0] + 6.0 * c[2]) - (t[0] - 6.0 * t[2]);
  const double s = (((lin ? dy * jl : 0.0) + (rin ? dy * jr : 0.0)) + (bin ? dx * jb : 0.0)) +
                   (tin ? dx * jt : 0.0);
  const double len = (((lin ? dy : 0.0) + (rin ? dy : 0.0)) + (bin ? dx : 0.0)) + (tin ? dx : 0.0);
  const double nrm = (fabs(c[0]) + 6.0 * fabs(c[1])) + 6.0 * fabs(c[2]);
  return fabs(s) > (h * len) * nrm;
}
__device__ __forceinline__ bool kxrcf2d(const double* c, const double* l, const double* r,
                                        const double* b, const double* t, double velx,
                                        double vely, double dx, double dy, double h) {
  return kxrcf2d_in(c, l, r, b, t, velx > 0.0, velx < 0.0, vely > 0.0, vely < 0.0, dx, dy, h);
}

// ------------------------------------------------------------------ Euler (gamma law)
// Row f of L and column f of R of the 2D characteristic fields in direction d (0: x,
// 1: y) at a cell-average state, one field at a time to keep register use low.  In
// (rho, normal momentum, tangential momentum, E) ordering the columns of R are
// (1, un - c, ut, H - un c), (1, un, ut, q^2/2), (0, 0, 1, ut), (1, un + c, ut, H + un c),
// and L = R^{-1} in closed form.
__device__ __forceinline__ void euler_eig2d_field(const double* U, double gam, int d, int f,
                                                  double* Lr, double* Rc) {
  const double rho = U[0];
  const double u = U[1] / rho, v = U[2] / rho, E = U[3];
  const double q2 = u * u + v * v;
  const double p = (gam - 1.0) * (E - 0.5 * rho * q2);
  const double c = sqrt(gam * p / rho);
  const double H = (E + p) / rho;
  const double b1 = (gam - 1.0) / (c * c), b2 = 0.5 * b1 * q2, ic = 1.0 / c;
  const double un = d == 0 ? u : v;   // normal velocity
  const double ut = d == 0 ? v : u;   // tangential velocity
  // in (normal, tangential) ordering of the momenta; mapped back below
  double l[4], r[4];
  if (f == 0) {
    l[0] = 0.5 * (b2 + un * ic); l[1] = -0.5 * (b1 * un + ic); l[2] = -0.5 * b1 * ut; l[3] = 0.5 * b1;
    r[0] = 1.0; r[1] = un - c; r[2] = ut; r[3] = H - un * c;
  } else if (f == 1) {
    l[0] = 1.0 - b2; l[1] = b1 * un; l[2] = b1 * ut; l[3] = -b1;
    r[0] = 1.0; r[1] = un; r[2] = ut; r[3] = 0.5 * q2;
  } else if (f == 2) {
    l[0] = -ut; l[1] = 0.0; l[2] = 1.0; l[3] = 0.0;
    r[0] = 0.0; r[1] = 0.0; r[2] = 1.0; r[3] = ut;
  } else {
    l[0] = 0.5 * (b2 - un * ic); l[1] = -0.5 * (b1 * un - ic); l[2] = -0.5 * b1 * ut; l[3] = 0.5 * b1;
    r[0] = 1.0; r[1] = un + c; r[2] = ut; r[3] = H + un * c;
  }
  // momentum index of the normal direction is 1 + d
  Lr[0] = l[0]; Lr[3] = l[3]; Rc[0] = r[0]; Rc[3] = r[3];
  if (d == 0) { Lr[1] = l[1]; Lr[2] = l[2]; Rc[1] = r[1]; Rc[2] = r[2]; }
  else { Lr[2] = l[1]; Lr[1] = l[2]; Rc[2] = r[1]; Rc[1] = r[2]; }
}

// physical flux of the scalar laws in direction d
template <int EQ>
__device__ __forceinline__ double scalar_flux(double u, double a) {
  if (EQ == EQ_ADV) return a * u;
  return 0.5 * u * u;
}

// Euler 1D flux (rho u, rho u^2 + p, u (E + p))
__device__ __forceinline__ void euler_flux1d(const double* U, double gam, double* f) {
  const double u = U[1] * rcp_nr(U[0]);
  const double p = (gam - 1.0) * (U[2] - 0.5 * U[1] * u);
  f[0] = U[1];
  f[1] = U[1] * u + p;
  f[2] = u * (U[2] + p);
}

// Euler 2D fluxes f (x) and g (y) at one point
__device__ __forceinline__ void euler_flux2d_x(const double* U, double gam, double* f) {
  const double r = rcp_nr(U[0]);
  const double u = U[1] * r, v = U[2] * r;
  const double p = (gam - 1.0) * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  f[0] = U[1];
  f[1] = U[1] * u + p;
  f[2] = U[2] * u;
  f[3] = u * (U[3] + p);
}
__device__ __forceinline__ void euler_flux2d_y(const double* U, double gam, double* g) {
  const double r = rcp_nr(U[0]);
  const double u = U[1] * r, v = U[2] * r;
  const double p = (gam - 1.0) * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  g[0] = U[2];
  g[1] = U[1] * v;
  g[2] = U[2] * v + p;
  g[3] = v * (U[3] + p);
}
__device__ __forceinline__ void euler_flux2d_xy(const double* U, double gam, double* f, double* g) {
  const double r = rcp_nr(U[0]);
  const double u = U[1] * r, v = U[2] * r;
  const double p = (gam - 1.0) * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  const double Ep = U[3] + p;
  f[0] = U[1];
  f[1] = U[1] * u + p;
  f[2] = U[2] * u;
  f[3] = u * Ep;
  g[0] = U[2];
  g[1] = U[1] * v;
  g[2] = U[2] * v + p;
  g[3] = v * Ep;
}

// The 2D characteristic decomposition in direction d (the matrices of euler_eig2d_field) as
// the lane of a four-lane group that works on characteristic field f and on physical
// component f needs it: row f of L (projection onto field f) and row f of R (component f
// of every field's eigenvector, for the way back).  Divisions by rho and c use rcp_nr.
__device__ __forceinline__ void euler_rows2d(const double* U, double gam, int d, int f,
                                             double* Lr, double* Rr) {
  const double ir = rcp_nr(U[0]);
  const double u = U[1] * ir, v = U[2] * ir, E = U[3];
  const double q2 = u * u + v * v;
  const double p = (gam - 1.0) * (E - 0.5 * U[0] * q2);
  const double c = sqrt(gam * p * ir);
  const double ic = rcp_nr(c);
  const double H = (E + p) * ir;
  const double b1 = (gam - 1.0) * (ic * ic), b2 = 0.5 * b1 * q2;
  const double un = d == 0 ? u : v, ut = d == 0 ? v : u;
  // row f of L in (rho, normal momentum, tangential momentum, E) ordering
  double l[4];
  if (f == 0) {
    l[0] = 0.5 * (b2 + un * ic); l[1] = -0.5 * (b1 * un + ic); l[2] = -0.5 * b1 * ut; l[3] = 0.5 * b1;
  } else if (f == 1) {
    l[0] = 1.0 - b2; l[1] = b1 * un; l[2] = b1 * ut; l[3] = -b1;
  } else if (f == 2) {
    l[0] = -ut; l[1] = 0.0; l[2] = 1.0; l[3] = 0.0;
  } else {
    l[0] = 0.5 * (b2 - un * ic); l[1] = -0.5 * (b1 * un - ic); l[2] = -0.5 * b1 * ut; l[3] = 0.5 * b1;
  }
  Lr[0] = l[0]; Lr[3] = l[3];
  Lr[1 + d] = l[1]; Lr[2 - d] = l[2];
  // row of R for physical component f (columns: fields 0..3)
  if (f == 0) {
    Rr[0] = 1.0; Rr[1] = 1.0; Rr[2] = 0.0; Rr[3] = 1.0;
  } else if (f == 3) {
    Rr[0] = H - un * c; Rr[1] = 0.5 * q2; Rr[2] = ut; Rr[3] = H + un * c;
  } else if (f == 1 + d) {   // normal momentum
    Rr[0] = un - c; Rr[1] = un; Rr[2] = 0.0; Rr[3] = un + c;
  } else {                   // tangential momentum
    Rr[0] = ut; Rr[1] = ut; Rr[2] = 1.0; Rr[3] = ut;
  }
}

// Every lane of each group of four consecutive lanes receives the four lanes' values of
// x (cross-lane moves within the group; all four lanes must be active).
__device__ __forceinline__ void quad_gather(double x, double* out) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
#define HW_QUAD_BCAST(g)                                                                   \
  out[g] = __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, (g) * 0x55, 0xF, 0xF, false), \
                            __builtin_amdgcn_update_dpp(0, lo, (g) * 0x55, 0xF, 0xF, false))
  HW_QUAD_BCAST(0);
  HW_QUAD_BCAST(1);
  HW_QUAD_BCAST(2);
  HW_QUAD_BCAST(3);
#undef HW_QUAD_BCAST
}

// spectral radius |velocity_d| + c at a cell average (Euler)
// spectral radii of both directions and the pressure, sharing one division
__device__ __forceinline__ void euler_speeds2d(const double* U, double gam, double& s0, double& s1,
                                               double& p) {
  const double r = 1.0 / U[0];
  const double u = U[1] * r, v = U[2] * r;
  p = (gam - 1.0) * (U[3] - 0.5 * (U[1] * u + U[2] * v));
  const double c = sqrt(gam * p * r);
  s0 = fabs(u) + c;
  s1 = fabs(v) + c;
}

}  // namespace hw

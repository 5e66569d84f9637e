// Reverse-mode building blocks of the stage operator of the hybrid Hermite WENO scheme
// (Zhao & Qiu, arXiv 2002.08816) with the troubled-cell flags, hybrid masks and
// Lax-Friedrichs speeds held fixed: the nonlinear weights (eqs. tao5 / tao4 and the
// weights below them), the Step-1 limiter of one first moment, and the edge values of
// Step 5.1.  Each recomputes the forward quantities it needs from the forward inputs and
// accumulates the cotangents of those inputs.  |x| inside tau is differentiated as
// sign(x), with sign(0) = 0.
#pragma once
#include "hw_tile2d.h"

namespace hw {

// Tiles plus halo (lx, ly in [lo, LX - lo)) of two [NF][ny][nx] arrays into LDS (b may be
// null; halo widths loa and lob), boundary conditions applied: transmissive ghosts mirror
// the cell and negate the normal moment.  Every global load of both is issued before any
// LDS store, so the tiles cost one memory round trip.
template <int NF, int NC>
__device__ __forceinline__ void load_tiles(const double* a, int loa, double* sa, const double* b,
                                           int lob, double* sb, int nx, int ny, int bcx, int bcy,
                                           int gx0, int gy0) {
  constexpr int NR = (LX * LX + NT - 1) / NT;   // positions per thread, at most
  const size_t plane = (size_t)nx * ny;
  double va[NR][NF], vb[NR][NF];
  int pa[NR], pb[NR];
  unsigned nga = 0, ngb = 0;   // bit 2 r: x moment negated, bit 2 r + 1: y moment negated
  auto fetch = [&](const double* in, int lo, double (*v)[NF], int* pos, unsigned& neg) {
    const int w = LX - 2 * lo;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int q = threadIdx.x + r * NT;
      pos[r] = -1;
      if (q < w * w) {
        const int ly = lo + q / w, lx = lo + q % w;
        pos[r] = ly * LX + lx;
        double sx, sy;
        const int gx = map_index(gx0 + lx, nx, bcx, sx);
        const int gy = map_index(gy0 + ly, ny, bcy, sy);
        if (sx < 0.0) neg |= 1u << (2 * r);
        if (sy < 0.0) neg |= 2u << (2 * r);
        const double* src = in + (size_t)gy * nx + gx;
#pragma unroll
        for (int f = 0; f < NF; ++f) v[r][f] = src[f * plane];
      }
    }
  };
  auto store = [&](double* s, double (*v)[NF], const int* pos, unsigned neg) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (pos[r] < 0) continue;
      const bool nxr = (neg >> (2 * r)) & 1u, nyr = (neg >> (2 * r + 1)) & 1u;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int m = f / NC;
        const bool ng = m == 1 ? nxr : (m == 2 ? nyr : false);
        s[f * NPOS + pos[r]] = ng ? -v[r][f] : v[r][f];
      }
    }
  };
  fetch(a, loa, va, pa, nga);
  if (b) fetch(b, lob, vb, pb, ngb);
  store(sa, va, pa, nga);
  if (b) store(sb, vb, pb, ngb);
}


__device__ __forceinline__ double sign0(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// beta-cotangents bb from omega-cotangents omb, for the weights
//   tau = (mean_n |beta_0 - beta_n|)^2, wbar_n = g_n (1 + tau / (beta_n + eps)),
//   omega_n = wbar_n / sum wbar.
template <int K>
__device__ __forceinline__ void nonlinear_weights_adj(const double* beta, const double* g, double eps,
                                                      const double* omb, double* bb) {
  double s = 0.0;
#pragma unroll
  for (int n = 1; n <= K; ++n) s += fabs(beta[0] - beta[n]);
  s = s / (double)K;
  const double tau = s * s;
  double wb[K + 1], r[K + 1], tot = 0.0;
#pragma unroll
  for (int n = 0; n <= K; ++n) {
    r[n] = 1.0 / (beta[n] + eps);
    wb[n] = g[n] * (1.0 + tau * r[n]);
    tot += wb[n];
  }
  // d omega_n / d wbar_m = (delta_nm - omega_n) / tot
  double dot = 0.0;
#pragma unroll
  for (int n = 0; n <= K; ++n) dot = fma(omb[n], wb[n], dot);
  dot = dot / tot;
  double taub = 0.0;
#pragma unroll
  for (int n = 0; n <= K; ++n) {
    const double wbb = (omb[n] - dot) / tot;
    taub = fma(wbb * g[n], r[n], taub);
    bb[n] = -wbb * g[n] * tau * r[n] * r[n];
  }
  const double sb = 2.0 * s * taub / (double)K;
#pragma unroll
  for (int n = 1; n <= K; ++n) {
    const double d = sign0(beta[0] - beta[n]) * sb;
    bb[0] += d;
    bb[n] -= d;
  }
}

// Cotangents (um, u0, up, vm, vp) of limit_moment's arguments for the cotangent vb of its
// result (Section 2.1 Step 1, the modified first moment).
__device__ __forceinline__ void limit_moment_adj(double um, double u0, double up, double vm, double vp,
                                                 const double* g, double eps, double vb, double* gb) {
  double q[3], t[5], b[3], om[3];
  limiter_terms(um, u0, up, vm, vp, q, t, b);
  nonlinear_weights<2>(b, g, eps, om);
  // value = om0 (q0/g0 - g1/g0 q1 - g2/g0 q2) + om1 q1 + om2 q2
  const double lin = q[0] / g[0] - g[1] / g[0] * q[1] - g[2] / g[0] * q[2];
  const double omb[3] = {vb * lin, vb * q[1], vb * q[2]};
  const double qb0 = vb * (om[0] / g[0]);
  const double qb1 = vb * (om[1] - om[0] * (g[1] / g[0]));
  const double qb2 = vb * (om[2] - om[0] * (g[2] / g[0]));
  double bb[3];
  nonlinear_weights_adj<2>(b, g, eps, omb, bb);
  const double tb1 = 2.0 * t[0] * bb[0];
  const double tb2 = 2.0 * t[1] * bb[0];
  const double tb3 = 2.0 * (3905.0 / 1444.0) * t[2] * bb[0];
  const double tb4 = 2.0 * (1.0 / 12.0) * t[3] * bb[0];
  const double tb5 = 2.0 * (109341.0 / 448.0) * t[4] * bb[0];
  const double d1 = 2.0 * (u0 - um) * bb[1];
  const double d2 = 2.0 * (up - u0) * bb[2];
  gb[0] = -(5.0 / 76.0) * qb0 - qb1 * (1.0 / 12.0) + (29.0 / 38.0) * tb1 + (9.0 / 4.0) * tb2 + tb3 +
          (5.0 / 2.0) * tb4 + tb5 - d1;
  gb[1] = (qb1 - qb2) * (1.0 / 12.0) - (9.0 / 2.0) * tb2 - 5.0 * tb4 - 2.0 * tb5 + d1 - d2;
  gb[2] = (5.0 / 76.0) * qb0 + qb2 * (1.0 / 12.0) - (29.0 / 38.0) * tb1 + (9.0 / 4.0) * tb2 - tb3 +
          (5.0 / 2.0) * tb4 + tb5 + d2;
  gb[3] = -(11.0 / 38.0) * qb0 + (60.0 / 19.0) * tb1 + (15.0 / 2.0) * tb2 + 12.0 * tb3 + 9.0 * tb4 +
          6.0 * tb5;
  gb[4] = -(11.0 / 38.0) * qb0 + (60.0 / 19.0) * tb1 - (15.0 / 2.0) * tb2 + 12.0 * tb3 - 9.0 * tb4 -
          6.0 * tb5;
}

// ------------------------------------------------------------------ linear maps, transposed
template <int NGE>
__device__ __forceinline__ void lin_edges_T(int dir, const double* ub, double* db) {
  if constexpr (NGE == 2) {
    if (dir == 0) hw2::lin2d_xedges_ng2_T(ub, db);
    else hw2::lin2d_yedges_ng2_T(ub, db);
  } else {
    if (dir == 0) hw2::lin2d_xedges_ng3_T(ub, db);
    else hw2::lin2d_yedges_ng3_T(ub, db);
  }
}
template <int NGE>
__device__ __forceinline__ void edge_quartic_T(double qb, int i, double* cb) {
  if constexpr (NGE == 2) hw2::edge_quartic_ng2_T(qb, i, cb);
  else hw2::edge_quartic_ng3_T(qb, i, cb);
}
template <int NGE>
__device__ __forceinline__ void edge_quad_T(double qb, int i, double* cb) {
  if constexpr (NGE == 2) hw2::edge_quad_ng2_T(qb, i, cb);
  else hw2::edge_quad_ng3_T(qb, i, cb);
}
template <int n>
__device__ __forceinline__ void pq_coeffs_T(const double* cb, double* db) {
  if constexpr (n == 1) hw2::p1_coeffs_T(cb, db);
  else if constexpr (n == 2) hw2::p2_coeffs_T(cb, db);
  else if constexpr (n == 3) hw2::p3_coeffs_T(cb, db);
  else hw2::p4_coeffs_T(cb, db);
}

// ------------------------------------------------------------------ Step 5.1, reversed
template <int NGE, int n>
__device__ __forceinline__ double hweno_pq_dot(const double* w19, int dir, const double* vb) {
  double c[6];
  pq_coeffs<n>(w19, c);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NGE; ++k) s = fma(vb[k], edge_quad<NGE>(c, dir * 2 * NGE + k), s);
  return s;
}
template <int NGE, int n>
__device__ __forceinline__ void hweno_pq_back(const double* w19, int dir, double an, double bbn,
                                              const double* vb, double* db) {
  double c[6], cb[6], gr[6];
  pq_coeffs<n>(w19, c);
#pragma unroll
  for (int t = 0; t < 6; ++t) cb[t] = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NGE; ++k) edge_quad_T<NGE>(an * vb[k], dir * 2 * NGE + k, cb);
  hw2::beta_pq_grad(c, gr);
#pragma unroll
  for (int t = 0; t < 6; ++t) cb[t] = fma(bbn, gr[t], cb[t]);
  pq_coeffs_T<n>(cb, db);
}

// Accumulates into db[19] the cotangent of the stencil w19 for the cotangents vb[2*NGE]
// of the edge values of direction dir (hweno2d_combine order); beta and om are the
// forward indicators and weights of this stencil (hweno2d_weights).
template <int NGE>
__device__ __forceinline__ void hweno2d_field_adj(const double* w19, const Weights& W, int dir,
                                                  const double* beta, const double* om,
                                                  const double* vb, double* db) {
  const double g0 = W.rec[0];
  double an[5];
  an[0] = om[0] / g0;
#pragma unroll
  for (int n = 1; n < 5; ++n) an[n] = om[n] - om[0] * (W.rec[n] / g0);
  // cotangents of the combination coefficients a_n
  double ab[5];
  {
    double c[15];
    hw2::p0_coeffs(w19, c);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * NGE; ++k) s = fma(vb[k], edge_quartic<NGE>(c, dir * 2 * NGE + k), s);
    ab[0] = s;
  }
  ab[1] = hweno_pq_dot<NGE, 1>(w19, dir, vb);
  ab[2] = hweno_pq_dot<NGE, 2>(w19, dir, vb);
  ab[3] = hweno_pq_dot<NGE, 3>(w19, dir, vb);
  ab[4] = hweno_pq_dot<NGE, 4>(w19, dir, vb);
  // a_0 = om_0 / g_0, a_n = om_n - om_0 g_n / g_0
  double omb[5];
  omb[0] = ab[0] / g0;
#pragma unroll
  for (int n = 1; n < 5; ++n) {
    omb[n] = ab[n];
    omb[0] -= ab[n] * (W.rec[n] / g0);
  }
  double bb[5];
  nonlinear_weights_adj<4>(beta, W.rec, W.eps, omb, bb);
  // candidates: through their edge values and their smoothness indicators
  {
    double c[15], cb[15], gr[15];
    hw2::p0_coeffs(w19, c);
#pragma unroll
    for (int t = 0; t < 15; ++t) cb[t] = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * NGE; ++k) edge_quartic_T<NGE>(an[0] * vb[k], dir * 2 * NGE + k, cb);
    hw2::beta_p0_grad(c, gr);
#pragma unroll
    for (int t = 0; t < 15; ++t) cb[t] = fma(bb[0], gr[t], cb[t]);
    hw2::p0_coeffs_T(cb, db);
  }
  hweno_pq_back<NGE, 1>(w19, dir, an[1], bb[1], vb, db);
  hweno_pq_back<NGE, 2>(w19, dir, an[2], bb[2], vb, db);
  hweno_pq_back<NGE, 3>(w19, dir, an[3], bb[3], vb, db);
  hweno_pq_back<NGE, 4>(w19, dir, an[4], bb[4], vb, db);
}

}  // namespace hw

// ================================================================== Euler (2D)
namespace hw {

// ub += (df/dU)^T fb + (dg/dU)^T gb for the two-dimensional Euler fluxes (eq. euler2)
// f = (m, m u + p, n u, u (E + p)) and g = (n, m v, n v + p, v (E + p)) at the point state
// U = (rho, m, n, E), with u = m / rho, v = n / rho, p = (gamma - 1)(E - (m u + n v) / 2).
__device__ __forceinline__ void euler_flux2d_vjp(const double* U, double gam, const double* fb,
                                                 const double* gb, double* ub) {
  const double r = 1.0 / U[0];
  const double m = U[1], n = U[2], E = U[3];
  const double u = m * r, v = n * r;
  const double p = (gam - 1.0) * (E - 0.5 * (m * u + n * v));
  const double Ep = E + p;
  double mb = fb[0] + fb[1] * u + gb[1] * v;
  double nb = gb[0] + fb[2] * u + gb[2] * v;
  double vu = fb[1] * m + fb[2] * n + fb[3] * Ep;   // cotangent of u
  double vv = gb[1] * m + gb[2] * n + gb[3] * Ep;   // cotangent of v
  const double Epb = fb[3] * u + gb[3] * v;
  const double pb = fb[1] + gb[2] + Epb;
  const double Eb = Epb + (gam - 1.0) * pb;
  const double Kb = -(gam - 1.0) * pb;               // K = (m u + n v) / 2
  mb += 0.5 * Kb * u;
  vu += 0.5 * Kb * m;
  nb += 0.5 * Kb * v;
  vv += 0.5 * Kb * n;
  mb += vu * r;
  nb += vv * r;
  const double rb = vu * m + vv * n;                 // cotangent of 1 / rho
  ub[0] += -rb * r * r;
  ub[1] += mb;
  ub[2] += nb;
  ub[3] += Eb;
}

// Forward-mode number (value, derivative along one seed direction).
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator+(double s, Dual a) { return {s + a.v, a.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}

// Derivatives of row f of L and column f of R (the characteristic matrices of
// euler_eig2d_field in direction d, Remark 4) with respect to the cell average U,
// contracted with cotangents: out[j] += sum_c Lb[c] dL[f][c]/dU_j + Rb[c] dR[c][f]/dU_j.
__device__ __forceinline__ void euler_eig2d_field_vjp(const double* U, double gam, int d, int f,
                                                      const double* Lb, const double* Rb,
                                                      double* out) {
  const Dual one{1.0, 0.0}, zero{0.0, 0.0};
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    const Dual rho{U[0], j == 0 ? 1.0 : 0.0}, M{U[1], j == 1 ? 1.0 : 0.0},
        N{U[2], j == 2 ? 1.0 : 0.0}, E{U[3], j == 3 ? 1.0 : 0.0};
    const Dual u = M / rho, v = N / rho;
    const Dual q2 = u * u + v * v;
    const Dual p = (gam - 1.0) * (E - 0.5 * (rho * q2));
    const Dual c = dsqrt((gam * p) / rho);
    const Dual H = (E + p) / rho;
    const Dual b1 = (gam - 1.0) * (one / (c * c)), b2 = 0.5 * (b1 * q2), ic = one / c;
    const Dual un = d == 0 ? u : v, ut = d == 0 ? v : u;
    Dual l[4], r[4];
    if (f == 0) {
      l[0] = 0.5 * (b2 + un * ic); l[1] = -0.5 * (b1 * un + ic); l[2] = -0.5 * (b1 * ut); l[3] = 0.5 * b1;
      r[0] = one; r[1] = un - c; r[2] = ut; r[3] = H - un * c;
    } else if (f == 1) {
      l[0] = one - b2; l[1] = b1 * un; l[2] = b1 * ut; l[3] = -b1;
      r[0] = one; r[1] = un; r[2] = ut; r[3] = 0.5 * q2;
    } else if (f == 2) {
      l[0] = -ut; l[1] = zero; l[2] = one; l[3] = zero;
      r[0] = zero; r[1] = zero; r[2] = one; r[3] = ut;
    } else {
      l[0] = 0.5 * (b2 - un * ic); l[1] = -0.5 * (b1 * un - ic); l[2] = -0.5 * (b1 * ut); l[3] = 0.5 * b1;
      r[0] = one; r[1] = un + c; r[2] = ut; r[3] = H + un * c;
    }
    // (normal, tangential) momentum ordering -> (x, y)
    const int in_ = 1 + d, it_ = 2 - d;
    double s = Lb[0] * l[0].d + Lb[3] * l[3].d + Rb[0] * r[0].d + Rb[3] * r[3].d;
    s += Lb[in_] * l[1].d + Lb[it_] * l[2].d + Rb[in_] * r[1].d + Rb[it_] * r[2].d;
    out[j] += s;
  }
}

// x[i] for a lane-dependent index i in 0..3
__device__ __forceinline__ double sel4(const double* x, int i) {
  return i == 0 ? x[0] : (i == 1 ? x[1] : (i == 2 ? x[2] : x[3]));
}

}  // namespace hw

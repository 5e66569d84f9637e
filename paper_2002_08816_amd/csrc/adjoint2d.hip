// Reverse pass of the two-dimensional stage operator for scalar conservation laws on
// periodic meshes (Zhao & Qiu, arXiv 2002.08816, Section 2.2 and eq. RK), with the
// troubled-cell flags, hybrid masks and Lax-Friedrichs speeds of the forward pass held
// fixed.  A stage is  W = Lim(u)  (Step 4),  out = a W(u^n) + b (W + dt L(W))  (eq. RK);
// its reverse is split in two kernels:
//
//  adjL2d   out = cg lam + cl (dL/dW)^T lam + ca acc.  The tile's stage input is staged
//           with three ghost layers, flags, limited moments and hybrid masks are re-derived
//           through the forward's own tile functions, and for every cell j of tile+1 the
//           cotangent d_j of its 19-value stencil is formed: the volume quadrature and the
//           four faces' Lax-Friedrichs fluxes give the cotangents of j's interior and edge
//           values (the flux is a sum of one term per side, so j's edge cotangents need
//           only j's own edge values and lam at j and its neighbours), which are pulled
//           back through the transposed linear maps (Step 5.2) or the reversed HWENO
//           combination (Step 5.1).  Then each tile cell gathers the entries of its
//           neighbours' d_j that refer to it: a scatter-free, deterministic transpose.
//  adjLim2d the transposed limiter Jacobian: every flagged cell of tile+1 differentiates
//           its two modified first moments with respect to their five inputs, and each
//           tile cell gathers what refers to it.
//
// Periodicity makes every LDS position a translate of a mesh cell, so a position's
// stencil cotangent equals that cell's and the gathers above are exact.
#include "hw_adjoint.h"

namespace hw {

template <int EQ>
__device__ __forceinline__ double dflux(double u, double a) {
  if constexpr (EQ == EQ_BURGERS) return u;
  else return a;
}

__device__ __forceinline__ int tq(int ly, int lx) { return (ly - 2) * R1 + (lx - 2); }

template <int EQ, int NGE>
__global__ __launch_bounds__(NT) void adjL2d_kernel(Adj2D P) {
  static_assert(EQ != EQ_EULER, "scalar equations only");
  constexpr int NQ = R1 * R1;                  // cells of tile+1
  __shared__ double s_in[3 * NPOS];            // stage input, then limited
  __shared__ double s_lam[3 * NPOS];           // lam on tile+2
  __shared__ double s_d[19 * NQ];              // stencil cotangents of tile+1
  __shared__ uint8_t s_T[NPOS];
  __shared__ uint8_t s_H[NPOS];
  __shared__ double s_alpha[2];

  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - HL, gy0 = by * TY - HL;
  const size_t plane = (size_t)nx * ny;

  reduce_speeds(P.alpha, s_alpha);
  load_tiles<3, 1>(P.in, 0, s_in, P.lam, 1, s_lam, nx, ny, BC_PERIODIC, BC_PERIODIC, gx0, gy0);
  __syncthreads();
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T);
  __syncthreads();
  if (P.tc_mode != TC_NONE) limit_tile<EQ>(s_in, s_T, 0.0, P.w);
  hybrid_tile(s_T, s_H);
  __syncthreads();

  const double ax = s_alpha[0], ay = s_alpha[1];
  const double idx = 1.0 / P.dx, idy = 1.0 / P.dy;
  const double* node = Gauss<NGE>::node;
  const double* wt = Gauss<NGE>::wt;

  for (int q = tid; q < NQ; q += NT) {
    const int ly = 2 + q / R1, lx = 2 + q % R1;
    double in19[19], d[19];
    gather19<1>(s_in, 0, ly, lx, in19);
#pragma unroll
    for (int k = 0; k < 19; ++k) d[k] = 0.0;
    const double lU = S(s_lam, 0, ly, lx);
    // volume terms of eq. ode2: the x moment gains (1/dx) sum w f(u(G)), the y moment
    // (1/dy) sum w g(u(G))
    {
      double inner[9], ub[9];
      hw2::lin2d_inner(in19, inner);
      const double lv = S(s_lam, 1, ly, lx) * idx, lw = S(s_lam, 2, ly, lx) * idy;
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        const double wq = VW[p % 3] * VW[p / 3];
        ub[p] = wq * (lv * dflux<EQ>(inner[p], P.adv0) + lw * dflux<EQ>(inner[p], P.adv1));
      }
      hw2::lin2d_inner_T(ub, d);
    }
    const bool hyb = s_H[ly * LX + lx] != 0;
    double beta[5], om[5];
    if (hyb) hweno2d_weights<NGE>(in19, P.w, beta, om);
#pragma unroll 1
    for (int dir = 0; dir < 2; ++dir) {
      const int oy = dir, ox = 1 - dir;
      const double inv = dir == 0 ? idx : idy;
      const double a = dir == 0 ? ax : ay;
      const double adv = dir == 0 ? P.adv0 : P.adv1;
      // the moment fed by (F_L + F_R)/2 and the one fed by the node-weighted difference
      const int fP = dir == 0 ? 1 : 2, fQ = 3 - fP;
      const double cP = S(s_lam, fP, ly, lx), cQ = S(s_lam, fQ, ly, lx);
      const double mU = S(s_lam, 0, ly - oy, lx - ox), mP = S(s_lam, fP, ly - oy, lx - ox),
                   mQ = S(s_lam, fQ, ly - oy, lx - ox);
      const double pU = S(s_lam, 0, ly + oy, lx + ox), pP = S(s_lam, fP, ly + oy, lx + ox),
                   pQ = S(s_lam, fQ, ly + oy, lx + ox);
      double v[2 * NGE];
      if (hyb) hweno2d_combine<NGE>(in19, P.w, dir, om, v);
      else lin_edges<NGE>(in19, dir, v, v + NGE);
      double ub[2 * NGE];
#pragma unroll
      for (int k = 0; k < NGE; ++k) {
        const double wk = wt[k] * inv, nk = node[k];
        // low face: this cell's left/bottom face and the neighbour's right/top face
        const double Flo = wk * ((lU - 0.5 * cP + nk * cQ) - (mU + 0.5 * mP + nk * mQ));
        // high face: this cell's right/top face and the neighbour's left/bottom face
        const double Fhi = wk * ((pU - 0.5 * pP + nk * pQ) - (lU + 0.5 * cP + nk * cQ));
        // F = (f(u-) + f(u+))/2 - a (u+ - u-)/2: this cell is u+ on the low face, u- on
        // the high face
        ub[k] = Flo * 0.5 * (dflux<EQ>(v[k], adv) - a);
        ub[NGE + k] = Fhi * 0.5 * (dflux<EQ>(v[NGE + k], adv) + a);
      }
      if (hyb) hweno2d_field_adj<NGE>(in19, P.w, dir, beta, om, ub, d);
      else lin_edges_T<NGE>(dir, ub, d);
    }
#pragma unroll
    for (int k = 0; k < 19; ++k) s_d[k * NQ + q] = d[k];
  }
  __syncthreads();

  // gather: slot k of cell j's stencil refers to cell j + offset_k
  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + HL, ly = ty + HL;
  const int gx = gx0 + lx, gy = gy0 + ly;
  if (gx >= nx || gy >= ny) return;
  double Wb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 9; ++k) Wb[0] += s_d[k * NQ + tq(ly - (k / 3 - 1), lx - (k % 3 - 1))];
  const int cy[5] = {-1, 0, 0, 0, 1}, cx[5] = {0, -1, 0, 1, 0};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    Wb[1] += s_d[(9 + k) * NQ + tq(ly - cy[k], lx - cx[k])];
    Wb[2] += s_d[(14 + k) * NQ + tq(ly - cy[k], lx - cx[k])];
  }
  const size_t gi = (size_t)gy * nx + gx;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double l = S(s_lam, f, ly, lx);
    double o = P.cg * l + P.cl * Wb[f];
    if (P.ca != 0.0) o = fma(P.ca, P.acc_in[f * plane + gi], o);
    P.out[f * plane + gi] = o;
    if (P.acc_mode == 1) P.acc_out[f * plane + gi] = P.kl * l;
    else if (P.acc_mode == 2) P.acc_out[f * plane + gi] = fma(P.kl, l, P.acc_in[f * plane + gi]);
  }
}

template <int EQ>
__global__ __launch_bounds__(NT) void adjLim2d_kernel(Adj2D P) {
  static_assert(EQ != EQ_EULER, "scalar equations only");
  constexpr int NQ = R1 * R1;
  __shared__ double s_in[3 * NPOS];
  __shared__ double s_g[3 * NPOS];     // cotangent of the limited input, tile+1
  __shared__ double s_c[10 * NQ];      // limiter partials of tile+1: x (um,u0,up,vm,vp), y
  __shared__ uint8_t s_T[NPOS];

  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - HL, gy0 = by * TY - HL;
  const size_t plane = (size_t)nx * ny;

  load_tiles<3, 1>(P.in, 0, s_in, P.lam, 2, s_g, nx, ny, BC_PERIODIC, BC_PERIODIC, gx0, gy0);
  __syncthreads();
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T);
  __syncthreads();
  const bool lim = P.tc_mode != TC_NONE;
  for (int q = tid; q < NQ; q += NT) {
    const int ly = 2 + q / R1, lx = 2 + q % R1;
    double gxv[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, gyv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (lim && s_T[ly * LX + lx]) {
      limit_moment_adj(S(s_in, 0, ly, lx - 1), S(s_in, 0, ly, lx), S(s_in, 0, ly, lx + 1),
                       S(s_in, 1, ly, lx - 1), S(s_in, 1, ly, lx + 1), P.w.lim, P.w.eps,
                       S(s_g, 1, ly, lx), gxv);
      limit_moment_adj(S(s_in, 0, ly - 1, lx), S(s_in, 0, ly, lx), S(s_in, 0, ly + 1, lx),
                       S(s_in, 2, ly - 1, lx), S(s_in, 2, ly + 1, lx), P.w.lim, P.w.eps,
                       S(s_g, 2, ly, lx), gyv);
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      s_c[m * NQ + q] = gxv[m];
      s_c[(5 + m) * NQ + q] = gyv[m];
    }
  }
  __syncthreads();

  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + HL, ly = ty + HL;
  const int gx = gx0 + lx, gy = gy0 + ly;
  if (gx >= nx || gy >= ny) return;
  const int qc = tq(ly, lx), qr = tq(ly, lx + 1), ql = tq(ly, lx - 1);
  const int qt = tq(ly + 1, lx), qb = tq(ly - 1, lx);
  const bool mine = lim && s_T[ly * LX + lx];
  // the right neighbour sees this cell as (um, vm), the left one as (up, vp)
  const double ub = S(s_g, 0, ly, lx) + s_c[1 * NQ + qc] + s_c[0 * NQ + qr] + s_c[2 * NQ + ql] +
                    s_c[6 * NQ + qc] + s_c[5 * NQ + qt] + s_c[7 * NQ + qb];
  const double vb = (mine ? 0.0 : S(s_g, 1, ly, lx)) + s_c[3 * NQ + qr] + s_c[4 * NQ + ql];
  const double wb = (mine ? 0.0 : S(s_g, 2, ly, lx)) + s_c[8 * NQ + qt] + s_c[9 * NQ + qb];
  const size_t gi = (size_t)gy * nx + gx;
  P.out[gi] = ub;
  P.out[plane + gi] = vb;
  P.out[2 * plane + gi] = wb;
}

}  // namespace hw

extern "C" hipError_t hw_launch_adj2d(int eq, int ng, const hw::Adj2D* P, hipStream_t s) {
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 block(hw::NT);
#define HW_LA(E, G) hipLaunchKernelGGL((hw::adjL2d_kernel<E, G>), grid, block, 0, s, *P)
  if (eq == hw::EQ_BURGERS && ng == 2) HW_LA(hw::EQ_BURGERS, 2);
  else if (eq == hw::EQ_BURGERS && ng == 3) HW_LA(hw::EQ_BURGERS, 3);
  else if (eq == hw::EQ_ADV && ng == 2) HW_LA(hw::EQ_ADV, 2);
  else if (eq == hw::EQ_ADV && ng == 3) HW_LA(hw::EQ_ADV, 3);
  else return hipErrorInvalidValue;
#undef HW_LA
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_adjlim2d(int eq, const hw::Adj2D* P, hipStream_t s) {
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 block(hw::NT);
  if (eq == hw::EQ_BURGERS)
    hipLaunchKernelGGL(hw::adjLim2d_kernel<hw::EQ_BURGERS>, grid, block, 0, s, *P);
  else if (eq == hw::EQ_ADV)
    hipLaunchKernelGGL(hw::adjLim2d_kernel<hw::EQ_ADV>, grid, block, 0, s, *P);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

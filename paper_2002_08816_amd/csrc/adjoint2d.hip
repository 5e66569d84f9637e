// Reverse pass of the two-dimensional stage operator (Zhao & Qiu, arXiv 2002.08816,
// Section 2.2 and eq. RK), with the troubled-cell flags, hybrid masks and Lax-Friedrichs
// speeds of the forward pass held fixed: scalar laws on meshes with periodic and
// transmissive sides, the Euler equations also with reflective sides and on the boundaries
// of Examples 3.10 and 3.11.  A stage is  W = Lim(u)  (Step 4),
// out = a W(u^n) + b (W + dt L(W))  (eq. RK).  For scalar conservation laws its reverse is
// split in two kernels (the Euler equations: five, further below):
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
// stencil cotangent equals that cell's and the gathers above are exact; at a transmissive
// side the ghosts mirror the cells beside it and their slots go back to those cells.
#include <climits>

#include "hw_adjoint.h"
#include "hw_dmr.h"
#include "hw_step.h"

namespace hw {

template <int EQ>
__device__ __forceinline__ double dflux(double u, double a) {
  if constexpr (EQ == EQ_BURGERS) return u;
  else return a;
}

__device__ __forceinline__ int tq(int ly, int lx) { return (ly - 2) * R1 + (lx - 2); }

// Transmissive sides (scalar laws): the LDS position (ly, lx) of the tile with origin
// (gx0, gy0) is a ghost when it lies beyond such a side; (my, mx) receives the LDS position
// of the mesh cell it mirrors, fx / fy whether it is mirrored in x / y.
__device__ __forceinline__ bool ghost_lds(const Adj2D& P, int gx0, int gy0, int ly, int lx, int& my,
                                          int& mx, bool& fx, bool& fy) {
  const int gx = gx0 + lx, gy = gy0 + ly;
  fx = P.bcx != BC_PERIODIC && (gx < 0 || gx >= P.nx);
  fy = P.bcy != BC_PERIODIC && (gy < 0 || gy >= P.ny);
  double s;
  mx = fx ? map_index(gx, P.nx, P.bcx, s) - gx0 : lx;
  my = fy ? map_index(gy, P.ny, P.bcy, s) - gy0 : ly;
  return fx || fy;
}

// The ghosts of [lo, LX - lo)^2 take the value of the cell they mirror in m (flags, hybrid
// masks), as in the forward stage.  A ghost's mirror is never a ghost.
__device__ __forceinline__ void mirror_ghost_bytes(const Adj2D& P, int gx0, int gy0, uint8_t* m, int lo) {
  const int w = LX - 2 * lo;
  for (int q = threadIdx.x; q < w * w; q += NT) {
    const int ly = lo + q / w, lx = lo + q % w;
    int my, mx;
    bool fx, fy;
    if (ghost_lds(P, gx0, gy0, ly, lx, my, mx, fx, fy)) m[ly * LX + lx] = m[my * LX + mx];
  }
}

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

  // transmissive sides: ghosts are staged as mirror images (moment normal to the side
  // negated) and take the flags of the cells they mirror; they carry no cotangent of their
  // own (lam = 0, no stencil cotangent).  A ghost's trace on the side is its cell's own
  // trace, so the ghost side of a wall face's flux is added to the wall cell's trace
  // cotangent, and slots of the wall cells' stencils that refer to a ghost go back to the
  // cell it mirrors in the gather
  const bool walls = P.bcx != BC_PERIODIC || P.bcy != BC_PERIODIC;
  reduce_speeds(P.alpha, s_alpha);
  load_tiles<3, 1>(P.in, 0, s_in, P.lam, 1, s_lam, nx, ny, P.bcx, P.bcy, gx0, gy0);
  __syncthreads();
  if (walls) {
    for (int q = tid; q < NPOS; q += NT) {
      int my, mx;
      bool fx, fy;
      if (ghost_lds(P, gx0, gy0, q / LX, q % LX, my, mx, fx, fy))
        s_lam[q] = s_lam[NPOS + q] = s_lam[2 * NPOS + q] = 0.0;
    }
  }
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T);
  __syncthreads();
  if (walls) {
    mirror_ghost_bytes(P, gx0, gy0, s_T, 1);
    __syncthreads();
  }
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
#pragma unroll
    for (int k = 0; k < 19; ++k) d[k] = 0.0;
    int wall = 0;   // bits: low x, high x, low y, high y face on a transmissive side
    if (walls) {
      int my, mx;
      bool fx, fy;
      if (ghost_lds(P, gx0, gy0, ly, lx, my, mx, fx, fy)) {
#pragma unroll
        for (int k = 0; k < 19; ++k) s_d[k * NQ + q] = 0.0;
        continue;
      }
      const int gxq = gx0 + lx, gyq = gy0 + ly;
      if (P.bcx != BC_PERIODIC) wall |= (gxq == 0 ? 1 : 0) | (gxq == nx - 1 ? 2 : 0);
      if (P.bcy != BC_PERIODIC) wall |= (gyq == 0 ? 4 : 0) | (gyq == ny - 1 ? 8 : 0);
    }
    gather19<1>(s_in, 0, ly, lx, in19);
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
        // a face on a transmissive side: the ghost's trace there is this cell's, so the
        // ghost side of the flux (u- on the low face, u+ on the high face) is this cell's
        if ((wall >> (2 * dir)) & 1) ub[k] += Flo * 0.5 * (dflux<EQ>(v[k], adv) + a);
        if ((wall >> (2 * dir + 1)) & 1) ub[NGE + k] += Fhi * 0.5 * (dflux<EQ>(v[NGE + k], adv) - a);
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
  if (walls) {
    // slots of the mesh cells' stencils that refer to a ghost mirroring this cell (one ghost
    // layer beside each transmissive side, and the corner between two; ghosts further out
    // belong to no mesh cell's stencil, and ghosts have no stencil cotangent)
    int xs[3] = {lx, INT_MIN, INT_MIN}, ys[3] = {ly, INT_MIN, INT_MIN};
    int nxs = 1, nys = 1;
    const int gcand[4] = {-1, -2, nx, nx + 1}, hcand[4] = {-1, -2, ny, ny + 1};
    for (int c = 0; c < 4; ++c) {
      double s;
      if (P.bcx != BC_PERIODIC && nxs < 3 && map_index(gcand[c], nx, P.bcx, s) == gx) xs[nxs++] = gcand[c] - gx0;
      if (P.bcy != BC_PERIODIC && nys < 3 && map_index(hcand[c], ny, P.bcy, s) == gy) ys[nys++] = hcand[c] - gy0;
    }
    auto inq = [](int y, int x) { return y >= 2 && y < LX - 2 && x >= 2 && x < LX - 2; };
    for (int a = 0; a < nys; ++a)
      for (int b = 0; b < nxs; ++b) {
        if (a == 0 && b == 0) continue;
        const int qy = ys[a], qx = xs[b];
        const double sx = b > 0 ? -1.0 : 1.0, sy = a > 0 ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const int py = qy - (k / 3 - 1), px = qx - (k % 3 - 1);
          if (inq(py, px)) Wb[0] += s_d[k * NQ + tq(py, px)];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int py = qy - cy[k], px = qx - cx[k];
          if (!inq(py, px)) continue;
          Wb[1] += sx * s_d[(9 + k) * NQ + tq(py, px)];
          Wb[2] += sy * s_d[(14 + k) * NQ + tq(py, px)];
        }
      }
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

  const bool walls = P.bcx != BC_PERIODIC || P.bcy != BC_PERIODIC;
  load_tiles<3, 1>(P.in, 0, s_in, P.lam, 2, s_g, nx, ny, P.bcx, P.bcy, gx0, gy0);
  __syncthreads();
  flags_tile<EQ>(s_in, P.tc_mode, P.adv0, P.adv1, P.dx, P.dy, P.h, s_T);
  __syncthreads();
  if (walls) {
    mirror_ghost_bytes(P, gx0, gy0, s_T, 1);
    __syncthreads();
  }
  const bool lim = P.tc_mode != TC_NONE;
  for (int q = tid; q < NQ; q += NT) {
    const int ly = 2 + q / R1, lx = 2 + q % R1;
    double gxv[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, gyv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int my, mx;
    bool fx, fy;
    // a ghost's limited moments are the mirror of its cell's: no limiter of its own
    const bool ghost = walls && ghost_lds(P, gx0, gy0, ly, lx, my, mx, fx, fy);
    if (lim && !ghost && s_T[ly * LX + lx]) {
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
  double vb = (mine ? 0.0 : S(s_g, 1, ly, lx)) + s_c[3 * NQ + qr] + s_c[4 * NQ + ql];
  double wb = (mine ? 0.0 : S(s_g, 2, ly, lx)) + s_c[8 * NQ + qt] + s_c[9 * NQ + qb];
  double ubw = 0.0;
  if (mine) {
    // beside a transmissive side this cell's own limiter reads the ghost mirroring it
    if (P.bcx != BC_PERIODIC && gx == 0) { ubw += s_c[0 * NQ + qc]; vb -= s_c[3 * NQ + qc]; }
    if (P.bcx != BC_PERIODIC && gx == nx - 1) { ubw += s_c[2 * NQ + qc]; vb -= s_c[4 * NQ + qc]; }
    if (P.bcy != BC_PERIODIC && gy == 0) { ubw += s_c[5 * NQ + qc]; wb -= s_c[8 * NQ + qc]; }
    if (P.bcy != BC_PERIODIC && gy == ny - 1) { ubw += s_c[7 * NQ + qc]; wb -= s_c[9 * NQ + qc]; }
  }
  const size_t gi = (size_t)gy * nx + gx;
  P.out[gi] = ub + ubw;
  P.out[plane + gi] = vb;
  P.out[2 * plane + gi] = wb;
}

// ================================================================== 2D Euler
// The reverse of a 2D Euler stage (eq. euler2) on a mesh with periodic, transmissive or
// reflective sides, with flags, hybrid masks and speeds held fixed.  The forward's own prepasses (flags and work lists, the limiter
// over the flagged list, HWENO over the hybrid list) are rerun on the stored stage input
// first, so the reverse sees the forward's decisions and values bit for bit; then:
//
//  adjEL2d    per tile cell j: the cotangents of j's nine interior values (volume
//             quadrature through the transposed flux Jacobians) and of its edge values
//             (the four faces' Lax-Friedrichs fluxes), pulled back through the transposed
//             linear maps (Step 5.2) to j's 4 x 19 stencil values.  For a hybrid cell only
//             the interior part; its edge cotangents are stored for the next pass.
//  adjEhw2d   over the hybrid list, four lanes per cell and direction (lane f:
//             characteristic field f and physical component f), the x and y directions in
//             the two waves of a pair: the reversed characteristic HWENO combination (Step
//             5.1, Remark 4), including the eigenvectors' dependence on the cell average,
//             added to the stencil cotangents.
//  adjEG2d    per cell: the gather of the stencil cotangents that refer to it,
//             out = cg lam + cl (dL/dW)^T lam + ca acc, and the running cotangent of u^n;
//  adjEC2d    over the forward's flagged list: the reversed characteristic limiter of both
//             directions (Step 4, Remark 4);
//  adjElim2d  per cell: the transposed limiter Jacobian (gathers of the flagged cells'
//             limiter cotangents that refer to it).
// A ghost position beside a transmissive or reflective side holds the mirrored cell's
// values; the kernels never form a ghost's own cotangent but add what refers to a ghost to
// the cell it mirrors (the instances for walls; periodic meshes use plain wrap-around).
// On the forward step, positions beyond the channel's sides and inside the step do the
// same with their source cell, and those beyond the inflow side hold the prescribed free
// stream, which carries no cotangent.

__device__ __forceinline__ int wrap(int g, int n) {
  double s;
  return map_index(g, n, BC_PERIODIC, s);
}

// The four values of a quad of lanes through ds_bpermute.  The reverse list kernels use it
// instead of the DPP quad moves of quad_gather: in several forms of these kernels (a
// run-time direction, mirrored stencil loads) the DPP moves returned values that were not
// the source lanes' with the compiler used here, while the same code through ds_bpermute
// agrees with the complex-step derivative of the oracle.
__device__ __forceinline__ void quad_gather_p(double x, double* out) {
  const int base = (int)(threadIdx.x & 63) & ~3;
#pragma unroll
  for (int g = 0; g < 4; ++g) out[g] = __shfl(x, base + g, 64);
}

// The Euler reverse on meshes with transmissive or reflective sides: a ghost position holds
// the values of the mesh cell it mirrors (Step 4's limiter and the stencils read it), with
// the moment normal to each side it lies beyond negated and, across a reflective side,
// the normal momentum too.  Its own cotangent is never formed: the reverse adds it to the
// cell it mirrors, through the same factors.
struct Mirror {
  int g;          // the mesh cell
  bool mx, my;    // mirrored across an x side / a y side
};
__device__ __forceinline__ Mirror mirror_of(const Adj2D& P, int gy, int gx) {
  double sx, sy;
  const int x = map_index(gx, P.nx, P.bcx, sx), y = map_index(gy, P.ny, P.bcy, sy);
  return {y * P.nx + x, sx < 0.0, sy < 0.0};
}
// factor of moment m (0 average, 1 x moment, 2 y moment) of component c at such a position
__device__ __forceinline__ double mirror_factor(const Adj2D& P, int m, int c, bool mx, bool my) {
  double f = 1.0;
  if (c == 1 && mx && P.bcx == BC_REFLECTIVE) f = -f;
  if (c == 2 && my && P.bcy == BC_REFLECTIVE) f = -f;
  if ((m == 1 && mx) || (m == 2 && my)) f = -f;
  return f;
}

// Boundary forms of the Euler reverse instances: periodic in both directions; a rectangle
// with a transmissive or reflective side (the mirrors above); and the resolver family: the
// forward step (Example 3.11), where a position outside the fluid -- beyond a side of the
// channel or inside the step -- takes the values of one fluid cell under the position rule
// of step::resolve, or the prescribed inflow state beyond the left side; the double Mach
// reflection (Example 3.10), whose positions right of the mesh mirror the outflow side,
// those below it from x = 1/6 on mirror the wall, and all others outside the mesh are
// prescribed (the stage's table of exact cut-cell moments).  Prescribed values carry no
// cotangent.
enum { ADJ_PERIODIC = 0, ADJ_WALLS = 1, ADJ_STEP = 2, ADJ_DMR = 3 };

__device__ __forceinline__ bool step_fluid(const Adj2D& P, int x, int y) {
  return x >= 0 && x < P.nx && y >= 0 && y < P.ny && !step::solid(x, y, P.si, P.sj);
}
// factor of moment m (0 average, 1 x moment, 2 y moment) of component c at a position
// whose source is r
__device__ __forceinline__ double step_factor(const step::Src& r, int m, int c) {
  const double w = step::comp_factor(r, c);
  return m == 0 ? w : (m == 1 ? r.sx * w : r.sy * w);
}
// The non-fluid side of face `side` (0 low, 1 high) of the fluid cell (gx, gy) in
// direction dir under the face rule: -2 a fluid cell or the prescribed inflow (no
// dependence on this cell's trace), -1 the outflow (this cell's own trace), 1 + dir a wall
// (the own trace with the normal momentum, component 1 + dir, reversed).
__device__ __forceinline__ int step_face(const Adj2D& P, int gx, int gy, int dir, int side) {
  const int qx = gx + (dir == 0 ? 2 * side - 1 : 0), qy = gy + (dir == 1 ? 2 * side - 1 : 0);
  if (step_fluid(P, qx, qy) || qx < 0) return -2;
  return qx >= P.nx ? -1 : 1 + dir;
}

// The double Mach reflection's position rule.  A prescribed position's values come from
// the stage's table by position (pres_value); its x, y are only clamped into the mesh.
__device__ __forceinline__ step::Src dmr_src(const Adj2D& P, int gx, int gy) {
  step::Src r{gx, gy, 1.0, 1.0, 1.0, 1.0, false};
  if (dmr::prescribed(gx, gy, P.nx, P.ny, P.x0, P.dx)) {
    r.pres = true;
    r.x = gx < 0 ? 0 : (gx >= P.nx ? P.nx - 1 : gx);
    r.y = gy < 0 ? 0 : (gy >= P.ny ? P.ny - 1 : gy);
    return r;
  }
  if (gx >= P.nx) {               // outflow: the even mirror
    r.x = 2 * P.nx - 1 - gx;
    r.sx = -1.0;
  }
  if (gy < 0) {                   // the wall: rho v reversed
    r.y = -1 - gy;
    r.sy = -1.0;
    r.fv = -1.0;
  }
  // positions beyond the ghost layers (partial tiles) are read by no mesh cell
  r.x = r.x < 0 ? 0 : (r.x >= P.nx ? P.nx - 1 : r.x);
  r.y = r.y < 0 ? 0 : (r.y >= P.ny ? P.ny - 1 : r.y);
  return r;
}
// the resolver family's source of a position, whether a mesh position is a fluid cell,
// field (m, c) of a prescribed position (gx, gy), and the non-fluid side of a face (the
// codes of step_face)
template <int BND>
__device__ __forceinline__ step::Src src_of(const Adj2D& P, int gx, int gy) {
  if constexpr (BND == ADJ_STEP) return step::resolve(gx, gy, P.nx, P.ny, P.si, P.sj);
  else return dmr_src(P, gx, gy);
}
template <int BND>
__device__ __forceinline__ bool fluid_of(const Adj2D& P, int x, int y) {
  if constexpr (BND == ADJ_STEP) return step_fluid(P, x, y);
  else return x >= 0 && x < P.nx && y >= 0 && y < P.ny;
}
template <int BND>
__device__ __forceinline__ double pres_value(const Adj2D& P, int m, int c, int gx, int gy) {
  if constexpr (BND == ADJ_STEP) return m == 0 ? sel4(P.uin, c) : 0.0;
  else return P.dtab[(size_t)(m * 4 + c) * dmr::ring2_size(P.nx, P.ny) + dmr::ring2_index(gx, gy, P.nx, P.ny)];
}
// whether every position within two cells of the fluid cell (gx, gy) is a fluid cell: then
// the cell is the source of no other position, and every slot that refers to it belongs to
// a fluid neighbour
template <int BND>
__device__ __forceinline__ bool interior_of(const Adj2D& P, int gx, int gy) {
  const bool in = gx >= 2 && gx <= P.nx - 3 && gy >= 2 && gy <= P.ny - 3;
  if constexpr (BND == ADJ_STEP) return in && !(gx >= P.si - 2 && gy <= P.sj + 1);
  else return in;
}
template <int BND>
__device__ __forceinline__ int face_of(const Adj2D& P, int gx, int gy, int dir, int side) {
  if constexpr (BND == ADJ_STEP) return step_face(P, gx, gy, dir, side);
  const int qx = gx + (dir == 0 ? 2 * side - 1 : 0), qy = gy + (dir == 1 ? 2 * side - 1 : 0);
  if (fluid_of<BND>(P, qx, qy) || dmr::prescribed(qx, qy, P.nx, P.ny, P.x0, P.dx)) return -2;
  return qx >= P.nx ? -1 : 1 + dir;
}
// The ghost's side of such a face, whose trace is this cell's own trace Uo with component
// cn reversed (cn = -1: none): the flux's derivative on that side, d/du- = (f' + a)/2 on
// the low face (side 0), d/du+ = (f' - a)/2 on the high face, with Fw half the face's
// weight, added to this cell's trace cotangent uo.
__device__ __forceinline__ void own_trace_face(int dir, int side, int cn, double a, double gam,
                                               const double* Fw, const double* Uo, double* uo) {
  constexpr int NC = 4;
  double Ug[NC], fg[NC], gg[NC], ug[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double r = c == cn ? -1.0 : 1.0;
    Ug[c] = r * Uo[c];
    fg[c] = dir == 0 ? Fw[c] : 0.0;
    gg[c] = dir == 0 ? 0.0 : Fw[c];
    ug[c] = (side == 0 ? a : -a) * Fw[c];
  }
  euler_flux2d_vjp(Ug, gam, fg, gg, ug);
#pragma unroll
  for (int c = 0; c < NC; ++c) uo[c] += (c == cn ? -1.0 : 1.0) * ug[c];
}

template <int NGE, int BND>
__global__ __launch_bounds__(NT) void adjEL2d_kernel(Adj2D P) {
  constexpr bool WALLS = BND == ADJ_WALLS;
  constexpr int NC = 4, NF = 12, W = TX + 2, NP = W * W;   // tile + one ghost layer
  __shared__ double s_w[NF * NP];    // limited stage input
  __shared__ double s_l[NF * NP];    // lam
  __shared__ double s_alpha[2];

  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  int bx, by;
  tile_of_block(nx, bx, by);
  const int gx0 = bx * TX - 1, gy0 = by * TY - 1;
  const size_t plane = (size_t)nx * ny;

  reduce_speeds(P.alpha, s_alpha);
  // ghost positions: the mirrored cell's values with their factors, and no cotangent of
  // their own (lam = 0: a ghost is not updated)
  for (int q = tid; q < NP; q += NT) {
    const int ly = q / W, lx = q - ly * W;
    if constexpr (BND >= ADJ_STEP) {
      const int px = gx0 + lx, py = gy0 + ly;
      const step::Src r = src_of<BND>(P, px, py);
      if (r.pres) {   // prescribed: never troubled, no cotangent
#pragma unroll
        for (int f = 0; f < NF; ++f) s_w[f * NP + q] = pres_value<BND>(P, f / NC, f % NC, px, py);
#pragma unroll
        for (int f = 0; f < NF; ++f) s_l[f * NP + q] = 0.0;
        continue;
      }
      const size_t g = (size_t)r.y * nx + r.x;
      const bool ghost = r.x != px || r.y != py;   // beyond a side or inside the step
      const bool t = P.T && P.T[g];
#pragma unroll
      for (int f = 0; f < NC; ++f) s_w[f * NP + q] = step_factor(r, 0, f) * P.in[f * plane + g];
#pragma unroll
      for (int f = NC; f < NF; ++f)
        s_w[f * NP + q] = step_factor(r, f / NC, f % NC) * (t ? P.lim[(f - NC) * plane + g] : P.in[f * plane + g]);
#pragma unroll
      for (int f = 0; f < NF; ++f) s_l[f * NP + q] = ghost ? 0.0 : P.lam[f * plane + g];
      continue;
    }
    if constexpr (BND == ADJ_PERIODIC) {
      const size_t g = (size_t)wrap(gy0 + ly, ny) * nx + wrap(gx0 + lx, nx);
      const bool t = P.T && P.T[g];
#pragma unroll
      for (int f = 0; f < NC; ++f) s_w[f * NP + q] = P.in[f * plane + g];
#pragma unroll
      for (int f = NC; f < NF; ++f) s_w[f * NP + q] = t ? P.lim[(f - NC) * plane + g] : P.in[f * plane + g];
#pragma unroll
      for (int f = 0; f < NF; ++f) s_l[f * NP + q] = P.lam[f * plane + g];
      continue;
    }
    const Mirror mr = mirror_of(P, gy0 + ly, gx0 + lx);
    const size_t g = (size_t)mr.g;
    const bool ghost = mr.mx || mr.my;
    const bool t = P.T && P.T[g];
#pragma unroll
    for (int f = 0; f < NC; ++f) s_w[f * NP + q] = mirror_factor(P, 0, f, mr.mx, mr.my) * P.in[f * plane + g];
#pragma unroll
    for (int f = NC; f < NF; ++f)
      s_w[f * NP + q] = mirror_factor(P, f / NC, f % NC, mr.mx, mr.my) *
                        (t ? P.lim[(f - NC) * plane + g] : P.in[f * plane + g]);
#pragma unroll
    for (int f = 0; f < NF; ++f) s_l[f * NP + q] = ghost ? 0.0 : P.lam[f * plane + g];
  }
  __syncthreads();

  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx + 1, ly = ty + 1;
  const int gx = bx * TX + tx, gy = by * TY + ty;
  if (gx >= nx || gy >= ny) return;   // no barrier below
  // the step's solid cells: no right-hand side (their stencil cotangents are never read)
  if constexpr (BND == ADJ_STEP) {
    if (step::solid(gx, gy, P.si, P.sj)) return;
  }
  const size_t gi = (size_t)gy * nx + gx;
  const bool hyb = P.H && P.H[gi];
  const double idx = 1.0 / P.dx, idy = 1.0 / P.dy;
  const double* node = Gauss<NGE>::node;
  const double* wt = Gauss<NGE>::wt;

  // volume terms of eq. ode2: the x moment gains (1/dx) sum w f(u(G)), the y moment
  // (1/dy) sum w g(u(G)); cotangents of the interior values
  double ubi[NC][9];
  {
    double inner[NC][9];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double in[19];
      gather19<NC, W>(s_w, c, ly, lx, in);
      hw2::lin2d_inner(in, inner[c]);
    }
    double lv[NC], lw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      lv[c] = S<W>(s_l, NC + c, ly, lx) * idx;
      lw[c] = S<W>(s_l, 2 * NC + c, ly, lx) * idy;
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const double wq = VW[p % 3] * VW[p / 3];
      double U[NC], fb[NC], gb[NC], ub[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        U[c] = inner[c][p];
        fb[c] = wq * lv[c];
        gb[c] = wq * lw[c];
        ub[c] = 0.0;
      }
      euler_flux2d_vjp(U, P.gam, fb, gb, ub);
#pragma unroll
      for (int c = 0; c < NC; ++c) ubi[c][p] = ub[c];
    }
  }

  // edge values of both directions and the cotangents of the four faces' fluxes
  double ube[2][NC][2 * NGE];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    double v[NC][2 * NGE];
    if (!hyb) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double in[19];
        gather19<NC, W>(s_w, c, ly, lx, in);
        lin_edges<NGE>(in, dir, v[c], v[c] + NGE);
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int k = 0; k < NGE; ++k) {
          v[c][k] = P.hwv[((((size_t)(dir * 2 + 0) * NGE + k) * NC + c)) * plane + gi];
          v[c][NGE + k] = P.hwv[((((size_t)(dir * 2 + 1) * NGE + k) * NC + c)) * plane + gi];
        }
    }
    const int oy = dir, ox = 1 - dir;
    const double inv = dir == 0 ? idx : idy;
    const double a = s_alpha[dir];
    // the moment fed by (F_L + F_R)/2 and the one fed by the node-weighted difference
    const int fP = dir == 0 ? 1 : 2, fQ = 3 - fP;
#pragma unroll
    for (int k = 0; k < NGE; ++k) {
      const double wk = wt[k] * inv, nk = node[k];
      double flo[NC], fhi[NC], zero[NC], ul[NC], uh[NC], Ul[NC], Uh[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double lU = S<W>(s_l, c, ly, lx), cP = S<W>(s_l, fP * NC + c, ly, lx),
                     cQ = S<W>(s_l, fQ * NC + c, ly, lx);
        const double mU = S<W>(s_l, c, ly - oy, lx - ox), mP = S<W>(s_l, fP * NC + c, ly - oy, lx - ox),
                     mQ = S<W>(s_l, fQ * NC + c, ly - oy, lx - ox);
        const double pU = S<W>(s_l, c, ly + oy, lx + ox), pP = S<W>(s_l, fP * NC + c, ly + oy, lx + ox),
                     pQ = S<W>(s_l, fQ * NC + c, ly + oy, lx + ox);
        // low face: this cell's left/bottom face and the neighbour's right/top face
        const double Flo = wk * ((lU - 0.5 * cP + nk * cQ) - (mU + 0.5 * mP + nk * mQ));
        // high face: this cell's right/top face and the neighbour's left/bottom face
        const double Fhi = wk * ((pU - 0.5 * pP + nk * pQ) - (lU + 0.5 * cP + nk * cQ));
        // F = (f(u-) + f(u+))/2 - a (u+ - u-)/2: this cell is u+ on the low face, u- on
        // the high face
        flo[c] = 0.5 * Flo;
        fhi[c] = 0.5 * Fhi;
        ul[c] = -0.5 * a * Flo;
        uh[c] = 0.5 * a * Fhi;
        zero[c] = 0.0;
        Ul[c] = v[c][k];
        Uh[c] = v[c][NGE + k];
      }
      if (dir == 0) {
        euler_flux2d_vjp(Ul, P.gam, flo, zero, ul);
        euler_flux2d_vjp(Uh, P.gam, fhi, zero, uh);
      } else {
        euler_flux2d_vjp(Ul, P.gam, zero, flo, ul);
        euler_flux2d_vjp(Uh, P.gam, zero, fhi, uh);
      }
      // a face on a transmissive or reflective side: the ghost's trace there is this
      // cell's own trace (the normal momentum reversed at a reflective side), so the
      // ghost's side of the flux, d/du- on the low face and d/du+ on the high face, also
      // belongs to this cell
      const int bc = dir == 0 ? P.bcx : P.bcy;
      if (WALLS && bc != BC_PERIODIC) {
        const int gd = dir == 0 ? gx : gy, nd = dir == 0 ? nx : ny;
        const int cn = bc == BC_REFLECTIVE ? 1 + dir : -1;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (side == 0 ? gd != 0 : gd != nd - 1) continue;
          double Ug[NC], fg[NC], gg[NC], ug[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double r = c == cn ? -1.0 : 1.0;
            const double Fw = side == 0 ? flo[c] : fhi[c];   // half the face's weight
            Ug[c] = r * (side == 0 ? Ul[c] : Uh[c]);
            fg[c] = dir == 0 ? Fw : 0.0;
            gg[c] = dir == 0 ? 0.0 : Fw;
            ug[c] = (side == 0 ? a : -a) * Fw;   // d/du- = (f' + a)/2, d/du+ = (f' - a)/2
          }
          euler_flux2d_vjp(Ug, P.gam, fg, gg, ug);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double r = c == cn ? -1.0 : 1.0;
            if (side == 0) ul[c] += r * ug[c];
            else uh[c] += r * ug[c];
          }
        }
      }
      // the resolver family: the face rule on faces towards a non-fluid position
      if constexpr (BND >= ADJ_STEP) {
        const int kl = face_of<BND>(P, gx, gy, dir, 0), kh = face_of<BND>(P, gx, gy, dir, 1);
        if (kl != -2) own_trace_face(dir, 0, kl, a, P.gam, flo, Ul, ul);
        if (kh != -2) own_trace_face(dir, 1, kh, a, P.gam, fhi, Uh, uh);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ube[dir][c][k] = ul[c];
        ube[dir][c][NGE + k] = uh[c];
      }
    }
  }

  // pull back to the stencil values, component by component
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double d[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) d[k] = 0.0;
    hw2::lin2d_inner_T(ubi[c], d);
    if (!hyb) {
      lin_edges_T<NGE>(0, ube[0][c], d);
      lin_edges_T<NGE>(1, ube[1][c], d);
    }
#pragma unroll
    for (int k = 0; k < 19; ++k) P.D[(size_t)(c * 19 + k) * plane + gi] = d[k];
  }
  if (hyb) {
#pragma unroll
    for (int dir = 0; dir < 2; ++dir)
#pragma unroll
      for (int k = 0; k < 2 * NGE; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          P.E[((size_t)(dir * 2 * NGE + k) * NC + c) * plane + gi] = ube[dir][c][k];
  }
}

// Reversed characteristic HWENO edge values of one hybrid cell in direction DIR (Step 5.1,
// Remark 4), four lanes per cell as in the forward pass: lane f projects onto field f with
// row f of L, reverses field f's reconstruction, and returns in ib the stencil cotangents
// of physical component f; the eigenvectors' dependence on the cell average enters through
// the average's cotangent.
template <int NGE, int DIR, int BND>
__device__ __forceinline__ void adjEhw2d_cell(const Adj2D& P, int gi, int f, double* ib) {
  constexpr int NC = 4, dir = DIR;
  constexpr bool WALLS = BND == ADJ_WALLS;
  const size_t plane = (size_t)P.nx * P.ny;
  const int gy = gi / P.nx, gx = gi - gy * P.nx;
  const int cross[5] = {1, 3, 4, 5, 7};
  // component f of the limited stencil (ghost positions: the mirrored cell's values)
  double in[19];
  if constexpr (BND >= ADJ_STEP) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int px = gx + k % 3 - 1, py = gy + k / 3 - 1;
      const step::Src r = src_of<BND>(P, px, py);
      in[k] = r.pres ? pres_value<BND>(P, 0, f, px, py)
                     : step_factor(r, 0, f) * P.in[f * plane + (size_t)r.y * P.nx + r.x];
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int k = cross[j];
      const int px = gx + k % 3 - 1, py = gy + k / 3 - 1;
      const step::Src r = src_of<BND>(P, px, py);
      if (r.pres) {
        in[9 + j] = pres_value<BND>(P, 1, f, px, py);
        in[14 + j] = pres_value<BND>(P, 2, f, px, py);
        continue;
      }
      const size_t g = (size_t)r.y * P.nx + r.x;
      const bool t = P.T[g] != 0;
      in[9 + j] = step_factor(r, 1, f) * (t ? P.lim[f * plane + g] : P.in[(NC + f) * plane + g]);
      in[14 + j] = step_factor(r, 2, f) * (t ? P.lim[(NC + f) * plane + g] : P.in[(2 * NC + f) * plane + g]);
    }
  } else if constexpr (BND == ADJ_PERIODIC) {
    int gb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) gb[k] = wrap(gy + k / 3 - 1, P.ny) * P.nx + wrap(gx + k % 3 - 1, P.nx);
#pragma unroll
    for (int k = 0; k < 9; ++k) in[k] = P.in[f * plane + gb[k]];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int g = gb[cross[j]];
      const bool t = P.T[g] != 0;
      in[9 + j] = t ? P.lim[f * plane + g] : P.in[(NC + f) * plane + g];
      in[14 + j] = t ? P.lim[(NC + f) * plane + g] : P.in[(2 * NC + f) * plane + g];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const Mirror mr = mirror_of(P, gy + k / 3 - 1, gx + k % 3 - 1);
      in[k] = mirror_factor(P, 0, f, mr.mx, mr.my) * P.in[f * plane + mr.g];
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int k = cross[j];
      const Mirror mr = mirror_of(P, gy + k / 3 - 1, gx + k % 3 - 1);
      const int g = mr.g;
      const bool t = P.T[g] != 0;
      in[9 + j] = mirror_factor(P, 1, f, mr.mx, mr.my) * (t ? P.lim[f * plane + g] : P.in[(NC + f) * plane + g]);
      in[14 + j] = mirror_factor(P, 2, f, mr.mx, mr.my) *
                   (t ? P.lim[(NC + f) * plane + g] : P.in[(2 * NC + f) * plane + g]);
    }
  }
  double U[4];
  quad_gather_p(in[4], U);   // the cell average
  double Lr[4], Rc[4], x[4];
  euler_eig2d_field(U, P.gam, dir, f, Lr, Rc);   // row f of L, column f of R
  double w19[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    quad_gather_p(in[k], x);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s = fma(Lr[c], x[c], s);
    w19[k] = s;
  }
  double beta[5], om[5], wv[2 * NGE];
  hweno2d_weights<NGE>(w19, P.w, beta, om);
  hweno2d_combine<NGE>(w19, P.w, dir, om, wv);
  // v_c = sum_f R[c][f] wv_f: the field's cotangent and column f of R-bar
  double wvb[2 * NGE], Rb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 2 * NGE; ++k) {
    quad_gather_p(P.E[((size_t)(dir * 2 * NGE + k) * NC + f) * plane + gi], x);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      s = fma(Rc[c], x[c], s);
      Rb[c] = fma(x[c], wv[k], Rb[c]);
    }
    wvb[k] = s;
  }
  double w19b[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) w19b[k] = 0.0;
  hweno2d_field_adj<NGE>(w19, P.w, dir, beta, om, wvb, w19b);
  // w_f = sum_c L[f][c] in_c: row f of L-bar, and component f's cotangent through
  // column f of L (lane g holds row g)
  double Lb[4] = {0.0, 0.0, 0.0, 0.0}, Lc[4];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    quad_gather_p(in[k], x);
#pragma unroll
    for (int c = 0; c < 4; ++c) Lb[c] = fma(w19b[k], x[c], Lb[c]);
  }
  {
    double q0[4], q1[4], q2[4], q3[4];
    quad_gather_p(Lr[0], q0);
    quad_gather_p(Lr[1], q1);
    quad_gather_p(Lr[2], q2);
    quad_gather_p(Lr[3], q3);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const double col[4] = {q0[g], q1[g], q2[g], q3[g]};
      Lc[g] = sel4(col, f);
    }
  }
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    quad_gather_p(w19b[k], x);
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < 4; ++g) s = fma(Lc[g], x[g], s);
    ib[k] = s;
  }
  // the eigenvectors' dependence on the average: summed over the four fields, lane f
  // keeps the derivative along component f
  double ev[4] = {0.0, 0.0, 0.0, 0.0};
  euler_eig2d_field_vjp(U, P.gam, dir, f, Lb, Rb, ev);
  double e0[4], e1[4], e2[4], e3[4];
  quad_gather_p(ev[0], e0);
  quad_gather_p(ev[1], e1);
  quad_gather_p(ev[2], e2);
  quad_gather_p(ev[3], e3);
  const double es[4] = {e0[0] + e0[1] + e0[2] + e0[3], e1[0] + e1[1] + e1[2] + e1[3],
                        e2[0] + e2[1] + e2[2] + e2[3], e3[0] + e3[1] + e3[2] + e3[3]};
  ib[4] += sel4(es, f);
}

// The hybrid list's reversed HWENO reconstruction: the waves of a workgroup form pairs, the
// two waves of a pair take the same 16 cells, one the x direction, the other the y
// direction, and the y wave hands its shares to the x wave through LDS, which adds both to
// the stencil cotangents.  The two directions thus run side by side.
template <int NGE, int BND>
__global__ __launch_bounds__(NT) void adjEhw2d_kernel(Adj2D P) {
  constexpr int NC = 4, CPW = 64 / NC, NPAIR = NT / 128;
  __shared__ double s_ib[NPAIR][19][64];
  const int ncell = P.lens ? (int)P.lens[3] : P.counts[1];
  if (ncell == 0) return;
  const size_t plane = (size_t)P.nx * P.ny;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, pr = wv >> 1, dir = wv & 1;
  const int f = lane % NC;
  // the loop's bounds are the workgroup's, so every wave meets both barriers
  for (long long base = (long long)blockIdx.x * NPAIR * CPW; base < ncell;
       base += (long long)gridDim.x * NPAIR * CPW) {
    const long long cell = base + pr * CPW + lane / NC;
    const bool on = cell < ncell;   // whole groups of four lanes
    double ib[19];
    int gi = 0;
    if (on) {
      gi = P.hlist[cell];
      if (dir == 0) {
        adjEhw2d_cell<NGE, 0, BND>(P, gi, f, ib);
      } else {
        adjEhw2d_cell<NGE, 1, BND>(P, gi, f, ib);
#pragma unroll
        for (int k = 0; k < 19; ++k) s_ib[pr][k][lane] = ib[k];
      }
    }
    __syncthreads();
    if (on && dir == 0) {
#pragma unroll
      for (int k = 0; k < 19; ++k) P.D[(size_t)(f * 19 + k) * plane + gi] += ib[k] + s_ib[pr][k][lane];
    }
    __syncthreads();
  }
}

// Gather of the stencil cotangents and the stage coefficients.
template <int BND>
__global__ __launch_bounds__(NT) void adjEG2d_kernel(Adj2D P) {
  constexpr int NC = 4, NF = 12;
  constexpr bool WALLS = BND == ADJ_WALLS;
  const int nx = P.nx, ny = P.ny;
  const size_t plane = (size_t)nx * ny;
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i >= plane) return;
  const int gy = (int)(i / nx), gx = (int)(i - (size_t)gy * nx);
  // slot k of cell j's stencil refers to the position j + offset_k; the positions that hold
  // this cell's values are the cell itself and, beside a transmissive or reflective side,
  // the ghosts that mirror it (at most one per side, and the corner between two)
  double Wb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) Wb[f] = 0.0;
  const int cy[5] = {-1, 0, 0, 0, 1}, cx[5] = {0, -1, 0, 1, 0};
  if constexpr (BND == ADJ_PERIODIC) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const size_t j = (size_t)wrap(gy - (k / 3 - 1), ny) * nx + wrap(gx - (k % 3 - 1), nx);
#pragma unroll
      for (int c = 0; c < NC; ++c) Wb[c] += P.D[(size_t)(c * 19 + k) * plane + j];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const size_t j = (size_t)wrap(gy - cy[k], ny) * nx + wrap(gx - cx[k], nx);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Wb[NC + c] += P.D[(size_t)(c * 19 + 9 + k) * plane + j];
        Wb[2 * NC + c] += P.D[(size_t)(c * 19 + 14 + k) * plane + j];
      }
    }
  }
  // the forward step: the positions that take this fluid cell's values are the cell itself
  // and the non-fluid positions whose source it is (at most two cells away in x, one in y);
  // slot k of a fluid cell j refers to the position j + offset_k
  if constexpr (BND >= ADJ_STEP) {
    if (fluid_of<BND>(P, gx, gy)) {
      // the cell's own position: the slots of its fluid neighbours, with every load issued
      // (a non-fluid owner's slot is read at this cell and not added)
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int ox = gx - (k % 3 - 1), oy = gy - (k / 3 - 1);
        const bool ok = fluid_of<BND>(P, ox, oy);
        const size_t j = ok ? (size_t)oy * nx + ox : i;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double v = P.D[(size_t)(c * 19 + k) * plane + j];
          Wb[c] += ok ? v : 0.0;
        }
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int ox = gx - cx[k], oy = gy - cy[k];
        const bool ok = fluid_of<BND>(P, ox, oy);
        const size_t j = ok ? (size_t)oy * nx + ox : i;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double v = P.D[(size_t)(c * 19 + 9 + k) * plane + j];
          const double w = P.D[(size_t)(c * 19 + 14 + k) * plane + j];
          Wb[NC + c] += ok ? v : 0.0;
          Wb[2 * NC + c] += ok ? w : 0.0;
        }
      }
      // near a boundary: the non-fluid positions whose source the cell is
      if (!interior_of<BND>(P, gx, gy))
      for (int ey = -2; ey <= 2; ++ey)
        for (int ex = -2; ex <= 2; ++ex) {
          const int qx = gx + ex, qy = gy + ey;
          if ((ex == 0 && ey == 0) || fluid_of<BND>(P, qx, qy)) continue;
          const step::Src r = src_of<BND>(P, qx, qy);
          if (r.pres || r.x != gx || r.y != gy) continue;
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            const int ox = qx - (k % 3 - 1), oy = qy - (k / 3 - 1);
            if (!fluid_of<BND>(P, ox, oy)) continue;
            const size_t j = (size_t)oy * nx + ox;
#pragma unroll
            for (int c = 0; c < NC; ++c) Wb[c] += step_factor(r, 0, c) * P.D[(size_t)(c * 19 + k) * plane + j];
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            const int ox = qx - cx[k], oy = qy - cy[k];
            if (!fluid_of<BND>(P, ox, oy)) continue;
            const size_t j = (size_t)oy * nx + ox;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              Wb[NC + c] += step_factor(r, 1, c) * P.D[(size_t)(c * 19 + 9 + k) * plane + j];
              Wb[2 * NC + c] += step_factor(r, 2, c) * P.D[(size_t)(c * 19 + 14 + k) * plane + j];
            }
          }
        }
    }
  }
  const bool wx = WALLS && P.bcx != BC_PERIODIC, wy = WALLS && P.bcy != BC_PERIODIC;
  if constexpr (WALLS) {
    // the cell's own position, every load issued: owners wrap across a periodic side; a
    // position beyond another side is no cell, its slot is read at this cell and not added
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      int oy = gy - (k / 3 - 1), ox = gx - (k % 3 - 1);
      bool ok = true;
      if (wy) ok = ok && oy >= 0 && oy < ny; else oy = wrap(oy, ny);
      if (wx) ok = ok && ox >= 0 && ox < nx; else ox = wrap(ox, nx);
      const size_t j = ok ? (size_t)oy * nx + ox : i;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double v = P.D[(size_t)(c * 19 + k) * plane + j];
        Wb[c] += ok ? v : 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      int oy = gy - cy[k], ox = gx - cx[k];
      bool ok = true;
      if (wy) ok = ok && oy >= 0 && oy < ny; else oy = wrap(oy, ny);
      if (wx) ok = ok && ox >= 0 && ox < nx; else ox = wrap(ox, nx);
      const size_t j = ok ? (size_t)oy * nx + ox : i;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double v = P.D[(size_t)(c * 19 + 9 + k) * plane + j];
        const double w = P.D[(size_t)(c * 19 + 14 + k) * plane + j];
        Wb[NC + c] += ok ? v : 0.0;
        Wb[2 * NC + c] += ok ? w : 0.0;
      }
    }
  }
  // the ghosts that mirror the cell, beside a transmissive or reflective side
  const int xs[3] = {gx, wx && gx == 0 ? -1 : INT_MIN, wx && gx == nx - 1 ? nx : INT_MIN};
  const int ys[3] = {gy, wy && gy == 0 ? -1 : INT_MIN, wy && gy == ny - 1 ? ny : INT_MIN};
  const bool edge = xs[1] != INT_MIN || xs[2] != INT_MIN || ys[1] != INT_MIN || ys[2] != INT_MIN;
  for (int a = 0; a < 3 && WALLS && edge; ++a) {
    if (ys[a] == INT_MIN) continue;
    for (int b = 0; b < 3; ++b) {
      if (xs[b] == INT_MIN || (a == 0 && b == 0)) continue;
      const int qy = ys[a], qx = xs[b];
      const bool mx = b > 0, my = a > 0;
      // the owner of slot (dy, dx) that refers to (qy, qx): a mesh cell, or none
      auto owner = [&](int dy, int dx, size_t& j) {
        int oy = qy - dy, ox = qx - dx;
        if (wy) { if (oy < 0 || oy >= ny) return false; } else oy = wrap(oy, ny);
        if (wx) { if (ox < 0 || ox >= nx) return false; } else ox = wrap(ox, nx);
        j = (size_t)oy * nx + ox;
        return true;
      };
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        size_t j;
        if (!owner(k / 3 - 1, k % 3 - 1, j)) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          Wb[c] += mirror_factor(P, 0, c, mx, my) * P.D[(size_t)(c * 19 + k) * plane + j];
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        size_t j;
        if (!owner(cy[k], cx[k], j)) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Wb[NC + c] += mirror_factor(P, 1, c, mx, my) * P.D[(size_t)(c * 19 + 9 + k) * plane + j];
          Wb[2 * NC + c] += mirror_factor(P, 2, c, mx, my) * P.D[(size_t)(c * 19 + 14 + k) * plane + j];
        }
      }
    }
  }
  double G[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const double l = P.lam[f * plane + i];
    double o = P.cg * l + P.cl * Wb[f];
    if (P.ca != 0.0) o = fma(P.ca, P.acc_in[f * plane + i], o);
    G[f] = o;
    P.gw[f * plane + i] = o;
    if (P.acc_mode == 1) P.acc_out[f * plane + i] = P.kl * l;
    else if (P.acc_mode == 2) P.acc_out[f * plane + i] = fma(P.kl, l, P.acc_in[f * plane + i]);
  }
}

// The reversed characteristic limiter (Step 4, Remark 4) of one flagged cell in direction
// DIR, four lanes per cell: lane f reverses the limiter of characteristic field f and
// stores the cotangents of physical component f of the five stencil values of the
// direction (u_{-1}, u_0, u_{+1}, v_{-1}, v_{+1}), with the eigenvectors' dependence on
// the average added to the centre slot.
template <int DIR, int BND>
__device__ __forceinline__ void adjEC2d_cell(const Adj2D& P, size_t i, int f) {
  constexpr int NC = 4, dir = DIR, mf = 1 + DIR;
  const int nx = P.nx, ny = P.ny;
  const size_t plane = (size_t)nx * ny;
  const int gy = (int)(i / nx), gx = (int)(i - (size_t)gy * nx);
  // the two neighbours along the direction (ghosts: the mirrored cell's values; beyond the
  // forward step's inflow side, the free stream with first moments zero)
  double xm, xp, wm_, wp_;
  if constexpr (BND >= ADJ_STEP) {
    const int xmx = gx - (dir == 0), xmy = gy - (dir == 1), xpx = gx + (dir == 0), xpy = gy + (dir == 1);
    const step::Src rm = src_of<BND>(P, xmx, xmy);
    const step::Src rp = src_of<BND>(P, xpx, xpy);
    const size_t jm = (size_t)rm.y * nx + rm.x, jp = (size_t)rp.y * nx + rp.x;
    xm = rm.pres ? pres_value<BND>(P, 0, f, xmx, xmy) : step_factor(rm, 0, f) * P.in[f * plane + jm];
    xp = rp.pres ? pres_value<BND>(P, 0, f, xpx, xpy) : step_factor(rp, 0, f) * P.in[f * plane + jp];
    wm_ = rm.pres ? pres_value<BND>(P, mf, f, xmx, xmy) : step_factor(rm, mf, f) * P.in[(mf * NC + f) * plane + jm];
    wp_ = rp.pres ? pres_value<BND>(P, mf, f, xpx, xpy) : step_factor(rp, mf, f) * P.in[(mf * NC + f) * plane + jp];
  } else {
    const Mirror mm = dir == 0 ? mirror_of(P, gy, gx - 1) : mirror_of(P, gy - 1, gx);
    const Mirror mp = dir == 0 ? mirror_of(P, gy, gx + 1) : mirror_of(P, gy + 1, gx);
    xm = mirror_factor(P, 0, f, mm.mx, mm.my) * P.in[f * plane + mm.g];
    xp = mirror_factor(P, 0, f, mp.mx, mp.my) * P.in[f * plane + mp.g];
    wm_ = mirror_factor(P, mf, f, mm.mx, mm.my) * P.in[(mf * NC + f) * plane + mm.g];
    wp_ = mirror_factor(P, mf, f, mp.mx, mp.my) * P.in[(mf * NC + f) * plane + mp.g];
  }
  // Jacobi: every input is the unlimited stage input; G is the cotangent of the limited
  // moment of this direction
  double Ui[4], um[4], up[4], vm[4], vp[4], G[4];
  quad_gather_p(P.in[f * plane + i], Ui);
  quad_gather_p(xm, um);
  quad_gather_p(xp, up);
  quad_gather_p(wm_, vm);
  quad_gather_p(wp_, vp);
  quad_gather_p(P.gw[(mf * NC + f) * plane + i], G);
  double Lr[4], Rc[4];
  euler_eig2d_field(Ui, P.gam, dir, f, Lr, Rc);
  double cm = 0.0, c0 = 0.0, cp = 0.0, wm = 0.0, wp = 0.0, wb = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cm = fma(Lr[c], um[c], cm);
    c0 = fma(Lr[c], Ui[c], c0);
    cp = fma(Lr[c], up[c], cp);
    wm = fma(Lr[c], vm[c], wm);
    wp = fma(Lr[c], vp[c], wp);
    wb = fma(Rc[c], G[c], wb);
  }
  const double vc = limit_moment(cm, c0, cp, wm, wp, P.w.lim, P.w.eps);
  double gbv[5];
  limit_moment_adj(cm, c0, cp, wm, wp, P.w.lim, P.w.eps, wb, gbv);
  double Lb[4], Rb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Lb[c] = gbv[0] * um[c] + gbv[1] * Ui[c] + gbv[2] * up[c] + gbv[3] * vm[c] + gbv[4] * vp[c];
    Rb[c] = G[c] * vc;
  }
  double ev[4] = {0.0, 0.0, 0.0, 0.0};
  euler_eig2d_field_vjp(Ui, P.gam, dir, f, Lb, Rb, ev);
  // component f: sums over the four fields (lane g of the quad holds field g)
  double Lc[4];
  {
    double q0[4], q1[4], q2[4], q3[4];
    quad_gather_p(Lr[0], q0);
    quad_gather_p(Lr[1], q1);
    quad_gather_p(Lr[2], q2);
    quad_gather_p(Lr[3], q3);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const double col[4] = {q0[g], q1[g], q2[g], q3[g]};
      Lc[g] = sel4(col, f);
    }
  }
  double e0[4], e1[4], e2[4], e3[4];
  quad_gather_p(ev[0], e0);
  quad_gather_p(ev[1], e1);
  quad_gather_p(ev[2], e2);
  quad_gather_p(ev[3], e3);
  const double es[4] = {e0[0] + e0[1] + e0[2] + e0[3], e1[0] + e1[1] + e1[2] + e1[3],
                        e2[0] + e2[1] + e2[2] + e2[3], e3[0] + e3[1] + e3[2] + e3[3]};
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double x[4];
    quad_gather_p(gbv[q], x);
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < 4; ++g) s = fma(Lc[g], x[g], s);
    if (q == 1) s += sel4(es, f);
    P.C[((size_t)(dir * 5 + q) * NC + f) * plane + i] = s;
  }
}

// The reversed limiter over the forward's flagged list: waves alternate between the x and
// the y direction of the same 16 cells.  BND: ADJ_STEP or ADJ_DMR for the resolver family,
// else the mirrors of mirror_of (which reduce to wrap-around on periodic sides).
template <int BND>
__global__ __launch_bounds__(NT) void adjEC2d_kernel(Adj2D P) {
  constexpr int NC = 4, CPW = 64 / NC;
  const int ncnt = P.lens ? (int)P.lens[0] : P.counts[0];
  const long long ngroup = ((long long)ncnt + CPW - 1) / CPW;   // waves per direction
  const int lane = threadIdx.x & 63, f = lane % NC;
  for (long long wq = ((long long)blockIdx.x * NT + threadIdx.x) >> 6; wq < 2 * ngroup;
       wq += ((long long)gridDim.x * NT) >> 6) {
    const long long cell = (wq >> 1) * CPW + lane / NC;
    if (cell >= ncnt) continue;   // whole groups of four lanes
    const size_t i = (size_t)P.flist[cell];
    if (wq & 1) adjEC2d_cell<1, BND>(P, i, f);
    else adjEC2d_cell<0, BND>(P, i, f);
  }
}

// The transposed limiter Jacobian: a flagged cell's limited moments replace its stored
// ones (their cotangent moves to the limiter's inputs); the limiter of a flagged cell
// reads the averages of the cell and its two neighbours along the direction and the
// neighbours' moments (slots um, u0, up, vm, vp).  BND as for adjEC2d_kernel.
template <int BND>
__global__ __launch_bounds__(NT) void adjElim2d_kernel(Adj2D P) {
  constexpr int NC = 4;
  const int nx = P.nx, ny = P.ny;
  const size_t plane = (size_t)nx * ny;
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i == 0 && P.counts) {   // the list passes are done: empty the lists for the next stage
    P.counts[0] = 0;
    P.counts[1] = 0;
  }
  if (i >= plane) return;
  const int gy = (int)(i / nx), gx = (int)(i - (size_t)gy * nx);
  double ou[NC], ov[NC], ow[NC];
  const bool ti = P.T && P.T[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    ou[c] = P.gw[c * plane + i];
    ov[c] = ti ? 0.0 : P.gw[(NC + c) * plane + i];
    ow[c] = ti ? 0.0 : P.gw[(2 * NC + c) * plane + i];
  }
  auto C = [&](int dir, int s, int c, size_t j) {
    return P.C[((size_t)(dir * 5 + s) * NC + c) * plane + j];
  };
  // the forward step: the limiter of a flagged fluid cell j reads the positions j -+ e_dir;
  // this fluid cell gathers what refers to itself and to the non-fluid positions whose
  // source it is (solid cells are never flagged and are nobody's source)
  if (BND >= ADJ_STEP && P.T && interior_of<BND>(P, gx, gy)) {
    // the plain gather: the cell's own slots and its four neighbours' (right / top see it
    // as (um, vm), left / bottom as (up, vp))
    if (ti) {
#pragma unroll
      for (int c = 0; c < NC; ++c) ou[c] += C(0, 1, c, i) + C(1, 1, c, i);
    }
    const size_t xr = i + 1, xl = i - 1, yt = i + nx, yb = i - nx;
    if (P.T[xr]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(0, 0, c, xr); ov[c] += C(0, 3, c, xr); }
    }
    if (P.T[xl]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(0, 2, c, xl); ov[c] += C(0, 4, c, xl); }
    }
    if (P.T[yt]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(1, 0, c, yt); ow[c] += C(1, 3, c, yt); }
    }
    if (P.T[yb]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(1, 2, c, yb); ow[c] += C(1, 4, c, yb); }
    }
  } else if (BND >= ADJ_STEP && P.T && fluid_of<BND>(P, gx, gy)) {
    if (ti) {
#pragma unroll
      for (int c = 0; c < NC; ++c) ou[c] += C(0, 1, c, i) + C(1, 1, c, i);
    }
    for (int ey = -2; ey <= 2; ++ey)
      for (int ex = -2; ex <= 2; ++ex) {
        const int qx = gx + ex, qy = gy + ey;
        step::Src r{gx, gy, 1.0, 1.0, 1.0, 1.0, false};
        if (ex != 0 || ey != 0) {
          if (fluid_of<BND>(P, qx, qy)) continue;
          r = src_of<BND>(P, qx, qy);
          if (r.pres || r.x != gx || r.y != gy) continue;
        }
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
          const int ux = dir == 0, uy = dir == 1;
          // the owner below q sees q as its (up, vp); the owner above, as its (um, vm)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int ox = s == 0 ? qx - ux : qx + ux, oy = s == 0 ? qy - uy : qy + uy;
            if (!fluid_of<BND>(P, ox, oy)) continue;
            const size_t j = (size_t)oy * nx + ox;
            if (!P.T[j]) continue;
            const int su = s == 0 ? 2 : 0, sv = s == 0 ? 4 : 3;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              ou[c] += step_factor(r, 0, c) * C(dir, su, c, j);
              const double v = step_factor(r, 1 + dir, c) * C(dir, sv, c, j);
              if (dir == 0) ov[c] += v;
              else ow[c] += v;
            }
          }
        }
      }
  }
  if (BND < ADJ_STEP && P.T) {
    if (ti) {
#pragma unroll
      for (int c = 0; c < NC; ++c) ou[c] += C(0, 1, c, i) + C(1, 1, c, i);
    }
    const bool wx = P.bcx != BC_PERIODIC, wy = P.bcy != BC_PERIODIC;
    const size_t xr = (size_t)gy * nx + wrap(gx + 1, nx), xl = (size_t)gy * nx + wrap(gx - 1, nx);
    const size_t yt = (size_t)wrap(gy + 1, ny) * nx + gx, yb = (size_t)wrap(gy - 1, ny) * nx + gx;
    // the right / top neighbour sees this cell as (um, vm), the left / bottom one as (up, vp)
    if (!(wx && gx == nx - 1) && P.T[xr]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(0, 0, c, xr); ov[c] += C(0, 3, c, xr); }
    }
    if (!(wx && gx == 0) && P.T[xl]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(0, 2, c, xl); ov[c] += C(0, 4, c, xl); }
    }
    if (!(wy && gy == ny - 1) && P.T[yt]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(1, 0, c, yt); ow[c] += C(1, 3, c, yt); }
    }
    if (!(wy && gy == 0) && P.T[yb]) {
#pragma unroll
      for (int c = 0; c < NC; ++c) { ou[c] += C(1, 2, c, yb); ow[c] += C(1, 4, c, yb); }
    }
    // beside a transmissive or reflective side, this cell's own limiter reads the ghost
    // that mirrors it as its neighbour across that side
    if (ti) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (wx && gx == 0) {
          ou[c] += mirror_factor(P, 0, c, true, false) * C(0, 0, c, i);
          ov[c] += mirror_factor(P, 1, c, true, false) * C(0, 3, c, i);
        }
        if (wx && gx == nx - 1) {
          ou[c] += mirror_factor(P, 0, c, true, false) * C(0, 2, c, i);
          ov[c] += mirror_factor(P, 1, c, true, false) * C(0, 4, c, i);
        }
        if (wy && gy == 0) {
          ou[c] += mirror_factor(P, 0, c, false, true) * C(1, 0, c, i);
          ow[c] += mirror_factor(P, 2, c, false, true) * C(1, 3, c, i);
        }
        if (wy && gy == ny - 1) {
          ou[c] += mirror_factor(P, 0, c, false, true) * C(1, 2, c, i);
          ow[c] += mirror_factor(P, 2, c, false, true) * C(1, 4, c, i);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    P.out[c * plane + i] = ou[c];
    P.out[(NC + c) * plane + i] = ov[c];
    P.out[(2 * NC + c) * plane + i] = ow[c];
  }
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

namespace {
// the reverse launches of one Euler stage for edge rule NGE and boundary form BND
template <int NGE, int BND>
void launch_adjE(const hw::Adj2D* P, dim3 grid, dim3 cells, hipStream_t s) {
  // the limiter kernels share one instance between periodic sides and mirrors
  constexpr int LB = BND >= hw::ADJ_STEP ? BND : hw::ADJ_WALLS;
  const dim3 block(hw::NT);
  hipLaunchKernelGGL((hw::adjEL2d_kernel<NGE, BND>), grid, block, 0, s, *P);
  if (P->counts) hipLaunchKernelGGL((hw::adjEhw2d_kernel<NGE, BND>), dim3(1024), block, 0, s, *P);
  hipLaunchKernelGGL(hw::adjEG2d_kernel<BND>, cells, block, 0, s, *P);
  if (P->T) hipLaunchKernelGGL(hw::adjEC2d_kernel<LB>, dim3(1024), block, 0, s, *P);
  hipLaunchKernelGGL(hw::adjElim2d_kernel<LB>, cells, block, 0, s, *P);
}
}  // namespace

extern "C" hipError_t hw_launch_adj2d_euler(int ng, const hw::Adj2D* P, hipStream_t s) {
  const size_t plane = (size_t)P->nx * P->ny;
  dim3 grid(((P->nx + hw::TX - 1) / hw::TX) * ((P->ny + hw::TY - 1) / hw::TY));
  dim3 cells((unsigned)((plane + hw::NT - 1) / hw::NT));
  const int bnd = P->bcx == hw::BC_STEP  ? hw::ADJ_STEP
                  : P->bcx == hw::BC_DMR ? hw::ADJ_DMR
                  : (P->bcx != hw::BC_PERIODIC || P->bcy != hw::BC_PERIODIC) ? hw::ADJ_WALLS
                                                                             : hw::ADJ_PERIODIC;
  if (bnd == hw::ADJ_DMR && !P->dtab) return hipErrorInvalidValue;
  if (ng == 2 && bnd == hw::ADJ_PERIODIC) launch_adjE<2, hw::ADJ_PERIODIC>(P, grid, cells, s);
  else if (ng == 2 && bnd == hw::ADJ_WALLS) launch_adjE<2, hw::ADJ_WALLS>(P, grid, cells, s);
  else if (ng == 2 && bnd == hw::ADJ_STEP) launch_adjE<2, hw::ADJ_STEP>(P, grid, cells, s);
  else if (ng == 2) launch_adjE<2, hw::ADJ_DMR>(P, grid, cells, s);
  // the periodic NG = 3 case takes the mirror instances (their mirrors reduce to wrap-around
  // on periodic sides): the plain-wrap tile kernel needs more registers than a wave has there
  else if (ng == 3 && bnd == hw::ADJ_PERIODIC) launch_adjE<3, hw::ADJ_WALLS>(P, grid, cells, s);
  else if (ng == 3 && bnd == hw::ADJ_WALLS) launch_adjE<3, hw::ADJ_WALLS>(P, grid, cells, s);
  else if (ng == 3 && bnd == hw::ADJ_STEP) launch_adjE<3, hw::ADJ_STEP>(P, grid, cells, s);
  else if (ng == 3) launch_adjE<3, hw::ADJ_DMR>(P, grid, cells, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

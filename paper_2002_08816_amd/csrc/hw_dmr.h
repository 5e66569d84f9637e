// Boundary data of the double Mach reflection problem (Zhao & Qiu, arXiv 2002.08816,
// Example 3.10, after Woodward and Colella): a Mach 10 shock in a gamma = 1.4 gas meets a
// reflecting wall at 60 degrees.  The wall runs along y = 0 from x = 1/6; at time t the
// shock is the line x = 1/6 + (y + 20 t)/sqrt(3), with gas at rest (rho, u, v, p) =
// (1.4, 0, 0, 1) ahead of it and (8, 8.25 cos 30, -8.25 sin 30, 116.5) behind it.
//
// Boundary treatment of a mesh of [x0, x1] x [y0, y1] (the paper's [0, 4] x [0, 1]):
//   prescribed ghost cells: left of the mesh, above it, and below it left of x = 1/6; they
//     hold the exact solution's moments at the stage's time, are never troubled, and their
//     trace on the boundary face is the exact state at the face's Gauss points;
//   below the mesh from x = 1/6 on: a reflective wall (mirror, rho v reversed);
//   right of the mesh: outflow (the transmissive mirror).
#pragma once
#include "hw_stage.h"

namespace hw {
namespace dmr {

constexpr double X_WALL = 1.0 / 6.0;
constexpr double SQ3 = 1.7320508075688772935274463415058723669;
constexpr double INV_SQ3 = 0.57735026918962576450914878050195745565;

// conserved states (rho, rho u, rho v, E) ahead of and behind the shock, gamma = 1.4
__device__ __forceinline__ void states(double gam, double* pre, double* post) {
  const double c30 = 0.86602540378443864676372317075293618347, s30 = 0.5;
  const double u = 8.25 * c30, v = -8.25 * s30;
  pre[0] = 1.4;
  pre[1] = 0.0;
  pre[2] = 0.0;
  pre[3] = 1.0 / (gam - 1.0);
  post[0] = 8.0;
  post[1] = 8.0 * u;
  post[2] = 8.0 * v;
  post[3] = 116.5 / (gam - 1.0) + 0.5 * 8.0 * (u * u + v * v);
}

// c(t): the region behind the shock is x - y / sqrt(3) < c(t)
__device__ __forceinline__ double offset(double t) { return X_WALL + 20.0 * t * INV_SQ3; }

// exact conserved state at the point (x, y)
__device__ __forceinline__ void point_state(double x, double y, double t, double gam, double* U) {
  double pre[4], post[4];
  states(gam, pre, post);
  const bool behind = x - y * INV_SQ3 < offset(t);
#pragma unroll
  for (int c = 0; c < 4; ++c) U[c] = behind ? post[c] : pre[c];
}

// Area and first moments (int xi, int eta) of the part of the reference square
// [-1/2, 1/2]^2 where xi - eta / sqrt(3) < d: the square clipped against the half-plane,
// then the shoelace formulas over the clipped polygon (at most five vertices).
__device__ __forceinline__ void clipped_moments(double d, double& A, double& Mx, double& My) {
  const double sx[4] = {-0.5, 0.5, 0.5, -0.5}, sy[4] = {-0.5, -0.5, 0.5, 0.5};
  double px[5], py[5];
  int n = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = (i + 1) & 3;
    const double fp = sx[i] - sy[i] * INV_SQ3 - d, fq = sx[j] - sy[j] * INV_SQ3 - d;
    if (fp < 0.0) {
      px[n] = sx[i];
      py[n] = sy[i];
      ++n;
    }
    if ((fp < 0.0) != (fq < 0.0)) {
      const double s = fp / (fp - fq);
      px[n] = sx[i] + s * (sx[j] - sx[i]);
      py[n] = sy[i] + s * (sy[j] - sy[i]);
      ++n;
    }
  }
  double a = 0.0, x = 0.0, y = 0.0;
  for (int i = 0; i < n; ++i) {
    const int j = i + 1 == n ? 0 : i + 1;
    const double cr = px[i] * py[j] - px[j] * py[i];
    a += cr;
    x += (px[i] + px[j]) * cr;
    y += (py[i] + py[j]) * cr;
  }
  if (n < 3) a = x = y = 0.0;
  A = 0.5 * a;
  Mx = x / 6.0;
  My = y / 6.0;
}

// Moment f (= m * 4 + c: average, x moment, y moment of component c) of the exact solution
// over the square cell of centre (xc, yc) and side h.
__device__ __forceinline__ double cell_value(int f, double xc, double yc, double h, double t,
                                             double gam) {
  double pre[4], post[4];
  states(gam, pre, post);
  const double d = (offset(t) - xc + yc * INV_SQ3) / h;
  double A, Mx, My;
  clipped_moments(d, A, Mx, My);
  const int m = f >> 2, c = f & 3;
  const double jump = post[c] - pre[c];
  if (m == 0) return pre[c] + A * jump;
  return (m == 1 ? Mx : My) * jump;
}

// whether the ghost position (gx, gy) of an nx x ny mesh is a prescribed cell
__device__ __forceinline__ bool prescribed(int gx, int gy, int nx, int ny, double x0, double dx) {
  if (gx < 0 || gy >= ny) return true;
  return gy < 0 && x0 + (gx + 0.5) * dx < X_WALL;
}

// The table of the prescribed ghosts of a stage (dmr_table_kernel): the ring of two ghost
// layers around the mesh -- rows gy = -2, -1 (gx = -2 .. nx + 1), rows gy = ny, ny + 1,
// then columns gx = -2, -1, nx, nx + 1 (gy = 0 .. ny - 1); field f of entry r at
// f * ring2_size + r.  Positions further out (the padding of a partial last tile, which no
// mesh cell's stencil reaches) read the nearest ring entry.
__host__ __device__ __forceinline__ int ring2_size(int nx, int ny) { return 4 * (nx + 4) + 4 * ny; }
__device__ __forceinline__ int ring2_index(int gx, int gy, int nx, int ny) {
  gx = min(max(gx, -2), nx + 1);
  gy = min(max(gy, -2), ny + 1);
  const int w = nx + 4;
  if (gy < 0) return (gy + 2) * w + gx + 2;
  if (gy >= ny) return (2 + gy - ny) * w + gx + 2;
  return 4 * w + (gx < 0 ? gx + 2 : 2 + gx - nx) * ny + gy;
}
__device__ __forceinline__ void ring2_position(int r, int nx, int ny, int& gx, int& gy) {
  const int w = nx + 4;
  if (r < 2 * w) {
    gy = r / w - 2;
    gx = r % w - 2;
  } else if (r < 4 * w) {
    gy = ny + (r - 2 * w) / w;
    gx = (r - 2 * w) % w - 2;
  } else {
    const int col = (r - 4 * w) / ny;
    gy = (r - 4 * w) % ny;
    gx = col < 2 ? col - 2 : nx + col - 2;
  }
}

// the time of a stage's input: the step's time t has already been advanced by dt when its
// stages run (stage inputs at t - dt, t, t - dt/2); an operator-only call uses t
__device__ __forceinline__ double stage_time(const double* t, double dt, int mode) {
  const double tn = *t;
  if (mode == MODE_RK1) return tn - dt;
  if (mode == MODE_RK3) return tn - 0.5 * dt;
  return tn;
}

}  // namespace dmr
}  // namespace hw

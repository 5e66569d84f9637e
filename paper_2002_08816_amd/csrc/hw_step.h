// Boundary data of the forward-facing step (Zhao & Qiu, arXiv 2002.08816, Example 3.11,
// after Woodward and Colella): a channel with an inflow on the left, an outflow on the
// right, reflective walls at the top and bottom, and a step -- the cells i >= si, j < sj
// of the rectangular mesh -- whose two faces are reflective walls.  The step's cells are
// solid: never updated, never flagged.
//
// Position rule (every value a stencil reads at a position outside the fluid): the
// position takes the values of one fluid cell, its source -- beyond the left side the
// prescribed inflow state (average; first moments zero; never troubled); beyond the right
// side the even mirror; beyond the top and bottom the wall mirror (rho v reversed); a
// position inside the step is then mirrored across the step face it lies closer to (the
// left face: rho u reversed; the top face: rho v reversed), across both on the diagonal.
// Each mirror across a vertical (horizontal) line negates the x (y) first moment.
//
// Face rule (traces): on a face between a fluid cell and any other position, the other
// side's trace is the fluid cell's own trace, with the normal momentum reversed at a wall
// (as it is at the outflow); on the inflow side it is the inflow state.
#pragma once
#include "hw_stage.h"

namespace hw {
namespace step {

// the source of position (gx, gy) under the position rule: mesh cell (x, y), moment
// factors sx, sy, momentum factors fu, fv; pres: the prescribed inflow state instead
struct Src {
  int x, y;
  double sx, sy, fu, fv;
  bool pres;
};

__device__ __forceinline__ bool solid(int gx, int gy, int si, int sj) { return gx >= si && gy < sj; }

__device__ __forceinline__ Src resolve(int gx, int gy, int nx, int ny, int si, int sj) {
  Src r{gx, gy, 1.0, 1.0, 1.0, 1.0, false};
  if (gx < 0) {
    r.x = 0;
    r.y = gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);
    r.pres = true;
    return r;
  }
  if (gx >= nx) {                 // outflow
    r.x = 2 * nx - 1 - gx;
    r.sx = -1.0;
  }
  if (gy < 0) {                   // bottom wall
    r.y = -1 - gy;
    r.sy = -1.0;
    r.fv = -1.0;
  } else if (gy >= ny) {          // top wall
    r.y = 2 * ny - 1 - gy;
    r.sy = -1.0;
    r.fv = -1.0;
  }
  // positions further out than the ghost layers (those of a partial tile on a mesh
  // narrower or lower than two tiles) are never read by a fluid cell: clamp them into the
  // mesh so that every load stays in bounds
  r.x = r.x < 0 ? 0 : (r.x >= nx ? nx - 1 : r.x);
  r.y = r.y < 0 ? 0 : (r.y >= ny ? ny - 1 : r.y);
  if (solid(r.x, r.y, si, sj)) {
    const int a = r.x - si, b = sj - 1 - r.y;   // cells from the left face, the top face
    if (a <= b) {
      r.x = 2 * si - 1 - r.x;
      r.sx = -r.sx;
      r.fu = -r.fu;
    }
    if (b <= a) {
      r.y = 2 * sj - 1 - r.y;
      r.sy = -r.sy;
      r.fv = -r.fv;
    }
  }
  return r;
}

// factor of component c (Euler: rho, rho u, rho v, E) under the source's mirrors
__device__ __forceinline__ double comp_factor(const Src& r, int c) {
  return c == 1 ? r.fu : (c == 2 ? r.fv : 1.0);
}

}  // namespace step
}  // namespace hw

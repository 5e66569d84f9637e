// Fused one-dimensional stage kernel of the hybrid Hermite WENO scheme
// (Zhao & Qiu, arXiv 2002.08816, Section 2.1, Steps 1-3 and eq. odeH).
//
// A workgroup (T threads, one per cell; T = 64, 128, 256 or 512) processes one tile of T
// cells of one instance: the tile plus three ghost layers is staged in LDS, then KXRCF flags
// (tile+2), the Step-1 limiter on flagged cells (Jacobi, characteristic-wise for Euler),
// the hybrid mask (tile+1), interface values (Step 2.2 linear or Step 2.1 HWENO) and
// interior Gauss-Lobatto values (Step 2.3), Lax-Friedrichs fluxes exchanged through
// LDS, the four-point Gauss-Lobatto volume term, and the TVD-RK3 stage combination.
//
// The same tile routine serves a single solver (one instance) and the batched form: many
// independent instances of different sizes, concatenated field by field, advanced by a
// persistent grid that walks an (instance, tile) work list.  Each instance has its own
// Lax-Friedrichs speed, time step and time.
#include "hw_mesh1d.h"

namespace hw {


constexpr int H1 = 3;   // ghost layers: flags on tile+2 read one more cell

// block-wide max over NW waves; red must hold NW doubles
template <int NW>
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) m = fmax(m, red[i]);
  return m;
}

// 1D Euler characteristic fields at a cell-average state, taken one field at a time: row f
// of L = R^{-1} and column f of R (R columns (1, u-c, H-uc), (1, u, u^2/2), (1, u+c, H+uc)).
// Only the derived quantities of the state stay live between fields.
struct Char1 {
  double u, c, H, b1, b2, ic;
};

__device__ __forceinline__ Char1 char1d(double rho, double m, double E, double gam) {
  Char1 k;
  k.u = m / rho;
  const double p = (gam - 1.0) * (E - 0.5 * rho * k.u * k.u);
  k.c = sqrt(gam * p / rho);
  k.H = (E + p) / rho;
  k.b1 = (gam - 1.0) / (k.c * k.c);
  k.b2 = 0.5 * k.b1 * k.u * k.u;
  k.ic = 1.0 / k.c;
  return k;
}

__device__ __forceinline__ void char1d_left(const Char1& k, int f, double* Lr) {
  if (f == 0) {
    Lr[0] = 0.5 * (k.b2 + k.u * k.ic);
    Lr[1] = -0.5 * (k.b1 * k.u + k.ic);
    Lr[2] = 0.5 * k.b1;
  } else if (f == 1) {
    Lr[0] = 1.0 - k.b2;
    Lr[1] = k.b1 * k.u;
    Lr[2] = -k.b1;
  } else {
    Lr[0] = 0.5 * (k.b2 - k.u * k.ic);
    Lr[1] = -0.5 * (k.b1 * k.u - k.ic);
    Lr[2] = 0.5 * k.b1;
  }
}

__device__ __forceinline__ void char1d_right(const Char1& k, int f, double* Rc) {
  Rc[0] = 1.0;
  if (f == 0) {
    Rc[1] = k.u - k.c;
    Rc[2] = k.H - k.u * k.c;
  } else if (f == 1) {
    Rc[1] = k.u;
    Rc[2] = 0.5 * k.u * k.u;
  } else {
    Rc[1] = k.u + k.c;
    Rc[2] = k.H + k.u * k.c;
  }
}

template <int EQ>
__device__ __forceinline__ void flux1d(const double* U, double gam, double a, double* f) {
  if constexpr (EQ == EQ_EULER) euler_flux1d(U, gam, f);
  else f[0] = scalar_flux<EQ>(U[0], a);
}

// NU: a single instance on cells of different sizes (per-cell tables, hw_mesh1d.h)
template <int EQ, int T1, bool NU>
__device__ void stage1d_tile(const Stage1D& P, int inst, int i0, double* s_in, double* s_face,
                             uint8_t* s_T, uint8_t* s_H, double* s_red) {
  constexpr int L1 = T1 + 2 * H1;
  constexpr int NC = (EQ == EQ_EULER) ? 3 : 1;
  constexpr int NF = 2 * NC;
  const int tid = threadIdx.x;
  const int mode = P.mode;
  double dt = 0.0;
  if (mode != MODE_L) {
    dt = P.dt[inst];
    if (dt == 0.0) return;   // uniform over the workgroup
  }
  const int off = P.off[inst], n = P.off[inst + 1] - off;
  const size_t tot = (size_t)P.total;
  // the cell an LDS position holds (a ghost: the cell it wraps to or mirrors) and its table
  auto tab = [&](int l) -> mesh1d::Tab {
    double sg;
    return mesh1d::Tab{P.nu, tot, off + map_index(i0 + l - H1, n, P.bc, sg)};
  };
  const double dx = NU ? tab(tid + H1)[mesh1d::K_DX] : P.dxs[inst];
  const double h = 0.5 * dx, idx = 1.0 / dx;

  // stage input -> LDS: positions tid and tid + T1 of the tile plus ghosts, every load
  // issued before the stores
  {
    double v0[NF], v1[NF], s0, s1;
    const int g0 = map_index(i0 + tid - H1, n, P.bc, s0);
    const bool two = tid + T1 < L1;
    const int g1 = two ? map_index(i0 + tid + T1 - H1, n, P.bc, s1) : 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) v0[f] = P.in[f * tot + off + g0];
    if (two) {
#pragma unroll
      for (int f = 0; f < NF; ++f) v1[f] = P.in[f * tot + off + g1];
    }
    // a reflective wall's ghost also negates the momentum (average and moment)
    const bool refl = EQ == EQ_EULER && P.bc == BC_REFLECTIVE;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double m = (refl && s0 < 0.0 && f % NC == 1) ? -1.0 : 1.0;
      s_in[f * L1 + tid] = m * (f >= NC ? s0 * v0[f] : v0[f]);
    }
    if (two) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double m = (refl && s1 < 0.0 && f % NC == 1) ? -1.0 : 1.0;
        s_in[f * L1 + tid + T1] = m * (f >= NC ? s1 * v1[f] : v1[f]);
      }
    }
  }
  __syncthreads();
  auto A = [&](int f, int l) -> double { return s_in[f * L1 + l]; };

  // At a transmissive or reflective boundary a ghost cell is the mirror image of the cell
  // it faces in every respect: the ghost next to the boundary takes that cell's flag and
  // its limited moments (under the state's sign rule), and its trace on the boundary face
  // is that cell's trace there.  Ghosts further out only feed values that are replaced.
  // mirror_src: the LDS position whose flag and limited moments the position l takes.
  const bool walls = P.bc != BC_PERIODIC;
  auto mirror_src = [&](int l) -> int {
    if (walls) {
      const int gl = i0 + l - H1;
      if (gl == -1) return l + 1;
      if (gl == n) return l - 1;
    }
    return l;
  };

  // ---------------------------------------------------------------- flags on tile+2
  for (int l = 1 + tid; l < L1 - 1; l += T1) {
    uint8_t t = 0;
    if (P.tc_mode == TC_ALL) {
      t = 1;
    } else if (P.tc_mode == TC_KXRCF) {
      const int lc = mirror_src(l);
      double vel;
      if constexpr (EQ == EQ_EULER) vel = A(1, lc) / A(0, lc);
      else if constexpr (EQ == EQ_BURGERS) vel = A(0, lc);
      else vel = P.adv;
      constexpr int ncheck = (EQ == EQ_EULER) ? 2 : 1;
      const double hl = NU ? 0.5 * tab(lc)[mesh1d::K_DX] : h;
      for (int k = 0; k < ncheck; ++k) {
        const int c = (k == 0) ? 0 : NC - 1;   // density, then energy
        if (kxrcf1d(A(c, lc), A(NC + c, lc), A(c, lc - 1), A(NC + c, lc - 1), A(c, lc + 1),
                    A(NC + c, lc + 1), vel, hl))
          t = 1;
      }
    }
    s_T[l] = t;
  }
  __syncthreads();

  // ---------------------------------------------------------------- limiter (Jacobi)
  double limv[2][NC];
  bool limdo[2] = {false, false};
  if (P.tc_mode != TC_NONE) {
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      const int lt = 1 + tid + rep * T1;
      if (lt >= L1 - 1) break;
      if (!s_T[lt]) continue;
      limdo[rep] = true;
      // the ghost next to a wall takes the mirror of its neighbour's limited moments
      const int l = mirror_src(lt);
      const bool mir = l != lt;
      if constexpr (EQ != EQ_EULER) {
        if constexpr (NU)
          limv[rep][0] = mesh1d::limit_moment_nu(tab(l), A(0, l - 1), A(0, l), A(0, l + 1),
                                                 A(1, l - 1), A(1, l + 1), P.w.lim, P.w.eps);
        else
          limv[rep][0] = limit_moment(A(0, l - 1), A(0, l), A(0, l + 1), A(1, l - 1), A(1, l + 1),
                                      P.w.lim, P.w.eps);
        if (mir) limv[rep][0] = -limv[rep][0];
      } else {
        // field by field: project, limit, and add R's column times the limited moment
        const Char1 k = char1d(A(0, l), A(1, l), A(2, l), P.gam);
#pragma unroll
        for (int c = 0; c < 3; ++c) limv[rep][c] = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          double Lr[3], Rc[3];
          char1d_left(k, f, Lr);
          double um = 0.0, u0 = 0.0, up = 0.0, vm = 0.0, vp = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            um = fma(Lr[c], A(c, l - 1), um);
            u0 = fma(Lr[c], A(c, l), u0);
            up = fma(Lr[c], A(c, l + 1), up);
            vm = fma(Lr[c], A(3 + c, l - 1), vm);
            vp = fma(Lr[c], A(3 + c, l + 1), vp);
          }
          double vc;
          if constexpr (NU) vc = mesh1d::limit_moment_nu(tab(l), um, u0, up, vm, vp, P.w.lim, P.w.eps);
          else vc = limit_moment(um, u0, up, vm, vp, P.w.lim, P.w.eps);
          char1d_right(k, f, Rc);
#pragma unroll
          for (int c = 0; c < 3; ++c) limv[rep][c] = fma(Rc[c], vc, limv[rep][c]);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (mir) {
          // first moments are odd under the mirror; a wall also reverses the momentum
          limv[rep][0] = -limv[rep][0];
          if (P.bc != BC_REFLECTIVE) limv[rep][1] = -limv[rep][1];
          limv[rep][2] = -limv[rep][2];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rep = 0; rep < 2; ++rep) {
    if (!limdo[rep]) continue;
    const int l = 1 + tid + rep * T1;
#pragma unroll
    for (int c = 0; c < NC; ++c) s_in[(NC + c) * L1 + l] = limv[rep][c];
  }
  for (int l = 2 + tid; l < L1 - 2; l += T1) s_H[l] = s_T[l - 1] | s_T[l] | s_T[l + 1];
  __syncthreads();

  // ---------------------------------------------------------------- reconstruction
  // interface values of cell l: left (u^+_{l-1/2}) and right (u^-_{l+1/2})
  auto traces = [&](int l, double* left, double* right, double* im, double* ip) {
    const bool hyb = s_H[l] != 0;
    // the HWENO branch first, so that no linear value is live across it
    if (hyb) {
      if constexpr (EQ != EQ_EULER) {
        if constexpr (NU) {
          const double d6[6] = {A(0, l - 1), A(0, l), A(0, l + 1), A(1, l - 1), A(1, l), A(1, l + 1)};
          mesh1d::hweno1d_nu(tab(l), d6, P.w.rec, P.w.eps, left[0], right[0]);
        } else {
          hweno1d(A(0, l - 1), A(0, l), A(0, l + 1), A(1, l - 1), A(1, l), A(1, l + 1), P.w.rec,
                  P.w.eps, left[0], right[0]);
        }
      } else {
        // field by field: project, reconstruct, and add R's column times the field's values
        const Char1 k = char1d(A(0, l), A(1, l), A(2, l), P.gam);
#pragma unroll
        for (int c = 0; c < 3; ++c) left[c] = right[c] = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          double Lr[3], Rc[3];
          char1d_left(k, f, Lr);
          double d[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d[0] = fma(Lr[c], A(c, l - 1), d[0]);
            d[1] = fma(Lr[c], A(c, l), d[1]);
            d[2] = fma(Lr[c], A(c, l + 1), d[2]);
            d[3] = fma(Lr[c], A(3 + c, l - 1), d[3]);
            d[4] = fma(Lr[c], A(3 + c, l), d[4]);
            d[5] = fma(Lr[c], A(3 + c, l + 1), d[5]);
          }
          double lf, rf;
          if constexpr (NU) mesh1d::hweno1d_nu(tab(l), d, P.w.rec, P.w.eps, lf, rf);
          else hweno1d(d[0], d[1], d[2], d[3], d[4], d[5], P.w.rec, P.w.eps, lf, rf);
          char1d_right(k, f, Rc);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            left[c] = fma(Rc[c], lf, left[c]);
            right[c] = fma(Rc[c], rf, right[c]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // linear values: the interface values of non-hybrid cells, the interior points of all
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double a, b, m, p;
      if constexpr (NU) {
        const double d6[6] = {A(c, l - 1), A(c, l), A(c, l + 1), A(NC + c, l - 1), A(NC + c, l),
                              A(NC + c, l + 1)};
        mesh1d::linear1d_nu(tab(l), d6, a, b, m, p);
      } else {
        linear1d(A(c, l - 1), A(c, l), A(c, l + 1), A(NC + c, l - 1), A(NC + c, l),
                 A(NC + c, l + 1), a, b, m, p);
      }
      if (!hyb) {
        left[c] = a;
        right[c] = b;
      }
      if (im) { im[c] = m; ip[c] = p; }
    }
  };

  const int l = tid + H1;
  const int gi = i0 + tid;
  const bool active = gi < n;
  // ---------------------------------------------------------------- face exchange
  // face q of the tile lies between cells q - 1 and q (q = 0..T1): u^- and u^+ there
  double* s_fm = s_face;             // u^- then the flux
  double* s_fp = s_face + NC * (T1 + 1);
  // ring cells first, in one pass of the last wave (the first wave takes the other extra
  // positions of the phases before and after): the left neighbour of the tile gives u^- at
  // face 0, the right neighbour u^+ at face T1
  if (tid >= T1 - 2) {
    const bool left_ring = tid == T1 - 2;
    double rL[NC], rR[NC];
    traces(left_ring ? H1 - 1 : H1 + T1, rL, rR, nullptr, nullptr);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (left_ring) s_fm[c * (T1 + 1)] = rR[c];
      else s_fp[c * (T1 + 1) + T1] = rL[c];
    }
  }
  double uL[NC], uR[NC], um[NC], up[NC];
  traces(l, uL, uR, um, up);
  const uint8_t myT = s_T[l];
  const uint8_t myH = s_H[l];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    s_fp[c * (T1 + 1) + tid] = uL[c];
    s_fm[c * (T1 + 1) + tid + 1] = uR[c];
  }
  __syncthreads();
  const double alpha = __longlong_as_double((long long)P.alpha_in[inst]);
  for (int q = tid; q < T1 + 1; q += T1) {
    double a[NC], b[NC], fa[NC], fb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      a[c] = s_fm[c * (T1 + 1) + q];
      b[c] = s_fp[c * (T1 + 1) + q];
    }
    if (walls) {
      // boundary face: the ghost's trace is the inner cell's (momentum reversed at a wall)
      const int gf = i0 + q;
      if (gf == 0 || gf == n) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double m = (EQ == EQ_EULER && P.bc == BC_REFLECTIVE && c == 1) ? -1.0 : 1.0;
          if (gf == 0) a[c] = m * b[c];
          else b[c] = m * a[c];
        }
      }
    }
    flux1d<EQ>(a, P.gam, P.adv, fa);
    flux1d<EQ>(b, P.gam, P.adv, fb);
#pragma unroll
    for (int c = 0; c < NC; ++c) s_fm[c * (T1 + 1) + q] = 0.5 * (fa[c] + fb[c]) - 0.5 * alpha * (b[c] - a[c]);
  }
  __syncthreads();
  double LU[NC], LV[NC];
  {
    double fL[NC], fR[NC], fm[NC], fp[NC];
    flux1d<EQ>(uL, P.gam, P.adv, fL);
    flux1d<EQ>(uR, P.gam, P.adv, fR);
    flux1d<EQ>(um, P.gam, P.adv, fm);
    flux1d<EQ>(up, P.gam, P.adv, fp);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double FL = s_fm[c * (T1 + 1) + tid], FR = s_fm[c * (T1 + 1) + tid + 1];
      const double Fi = (fL[c] + fR[c]) * (1.0 / 12.0) + (fm[c] + fp[c]) * (5.0 / 12.0);
      LU[c] = -(FR - FL) * idx;
      LV[c] = (Fi - 0.5 * (FL + FR)) * idx;
    }
  }
  double own[NF];   // the (limited) stage input
#pragma unroll
  for (int f = 0; f < NF; ++f) own[f] = A(f, l);
  __syncthreads();   // the LDS is reused by the next work item

  // ---------------------------------------------------------------- epilogue
  double sp = 0.0;
  if (active) {
    const size_t gidx = (size_t)off + gi;
    if (P.flagsT) P.flagsT[gidx] = myT;
    if (P.flagsH) P.flagsH[gidx] = myH;
    if (mode == MODE_L) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        P.out[c * tot + gidx] = LU[c];
        P.out[(NC + c) * tot + gidx] = LV[c];
      }
      if (P.wout) {
#pragma unroll
        for (int f = 0; f < NF; ++f) P.wout[f * tot + gidx] = own[f];
      }
    } else {
      double Wn[NF];
      if (mode == MODE_RK1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) Wn[f] = own[f];
        P.Tn[gidx] = myT;
        if (myT) {
#pragma unroll
          for (int c = 0; c < NC; ++c) P.limn[c * tot + gidx] = own[NC + c];
        }
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) Wn[f] = P.base[f * tot + gidx];
        if (P.Tn[gidx]) {
#pragma unroll
          for (int c = 0; c < NC; ++c) Wn[NC + c] = P.limn[c * tot + gidx];
        }
      }
      double res[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double Lf = f < NC ? LU[f] : LV[f - NC];
        double v;
        if (mode == MODE_RK1) v = own[f] + dt * Lf;
        else if (mode == MODE_RK2) v = (0.75 * Wn[f] + 0.25 * own[f]) + (0.25 * dt) * Lf;
        else v = (Wn[f] * (1.0 / 3.0) + (2.0 / 3.0) * own[f]) + ((2.0 / 3.0) * dt) * Lf;
        res[f] = v;
      }
      int bad = 0;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        P.out[f * tot + gidx] = res[f];
        if (!isfinite(res[f])) bad |= 1;
      }
      if constexpr (EQ == EQ_EULER) {
        const double ir = rcp_nr(res[0]), u = res[1] * ir;
        const double p = (P.gam - 1.0) * (res[2] - 0.5 * res[1] * u);
        if (!(res[0] > 0.0) || !(p > 0.0)) bad |= 2;
        sp = fabs(u) + sqrt(P.gam * p * ir);
      } else if constexpr (EQ == EQ_BURGERS) {
        sp = fabs(res[0]);
      } else {
        sp = fabs(P.adv);
      }
      if (bad) atomicOr(P.status, bad);
    }
  }
  if (mode != MODE_L) {
    const double m = block_max<T1 / 64>(sp, s_red);
    if (tid == 0) atomic_max_pos(&P.alpha_out[inst], m);
    __syncthreads();
  }
}

template <int EQ, int T1, bool NU>
__global__ __launch_bounds__(T1) void stage1d_kernel(Stage1D P) {
  constexpr int NF = (EQ == EQ_EULER) ? 6 : 2, L1 = T1 + 2 * H1;
  __shared__ double s_in[NF * L1];
  __shared__ double s_face[2 * NF / 2 * (T1 + 1)];
  __shared__ uint8_t s_T[L1], s_H[L1];
  __shared__ double s_red[T1 / 64];
  const int2 it = P.items[blockIdx.x];
  stage1d_tile<EQ, T1, NU>(P, it.x, it.y, s_in, s_face, s_T, s_H, s_red);
}

// persistent form: a grid sized to the machine walks the work list
template <int EQ, int T1>
__global__ __launch_bounds__(T1, 4) void stage1d_persistent(Stage1D P) {
  constexpr int NF = (EQ == EQ_EULER) ? 6 : 2, L1 = T1 + 2 * H1;
  __shared__ double s_in[NF * L1];
  __shared__ double s_face[2 * NF / 2 * (T1 + 1)];
  __shared__ uint8_t s_T[L1], s_H[L1];
  __shared__ double s_red[T1 / 64];
  for (int item = blockIdx.x; item < P.nitems; item += gridDim.x) {
    const int2 it = P.items[item];
    stage1d_tile<EQ, T1, false>(P, it.x, it.y, s_in, s_face, s_T, s_H, s_red);
  }
}

// Lax-Friedrichs speed per instance (before the first stage; operator-only calls)
template <int EQ>
__global__ __launch_bounds__(256) void alpha1d_kernel(const double* U, const int* off, int total,
                                                      double gam, double adv,
                                                      unsigned long long* alpha_out) {
  __shared__ double s_red[4];
  const int inst = blockIdx.y;
  const int o = off[inst], n = off[inst + 1] - o;
  double m = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    if constexpr (EQ == EQ_EULER) {
      const double rho = U[o + i], mom = U[(size_t)total + o + i], E = U[2 * (size_t)total + o + i];
      const double p = (gam - 1.0) * (E - mom * mom / (2.0 * rho));
      m = fmax(m, fabs(mom / rho) + sqrt(gam * p / rho));
    } else if constexpr (EQ == EQ_BURGERS) {
      m = fmax(m, fabs(U[o + i]));
    } else {
      m = fabs(adv);
    }
  }
  const double r = block_max256(m, s_red);
  if (threadIdx.x == 0) atomic_max_pos(&alpha_out[inst], r);
}

// ------------------------------------------------------------------ mesh tables
namespace mesh1d {

__device__ __forceinline__ double ipow(double x, int m) {
  double r = 1.0;
  for (int k = 0; k < m; ++k) r *= x;
  return r;
}

// int_lo^hi xi^m dxi
__device__ __forceinline__ double imono(int m, double lo, double hi) {
  return (ipow(hi, m + 1) - ipow(lo, m + 1)) / (m + 1);
}

// Condition row entry m: average (kind 0) or first moment (kind 1) of xi^m over the cell of
// centre c and width w
__device__ __forceinline__ double cond(int kind, double c, double w, int m) {
  const double lo = c - 0.5 * w, hi = c + 0.5 * w;
  if (kind == 0) return imono(m, lo, hi) / w;
  return (imono(m + 1, lo, hi) - c * imono(m, lo, hi)) / (w * w);
}

// Inverse of the N x N matrix A (row-major; destroyed) by Gauss-Jordan elimination with
// partial pivoting
template <int N>
__device__ void invert(double* A, double* X) {
  for (int r = 0; r < N; ++r)
    for (int c = 0; c < N; ++c) X[r * N + c] = r == c ? 1.0 : 0.0;
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int r = k + 1; r < N; ++r)
      if (fabs(A[r * N + k]) > fabs(A[piv * N + k])) piv = r;
    if (piv != k)
      for (int c = 0; c < N; ++c) {
        double t = A[k * N + c]; A[k * N + c] = A[piv * N + c]; A[piv * N + c] = t;
        t = X[k * N + c]; X[k * N + c] = X[piv * N + c]; X[piv * N + c] = t;
      }
    const double ip = 1.0 / A[k * N + k];
    for (int c = 0; c < N; ++c) {
      A[k * N + c] *= ip;
      X[k * N + c] *= ip;
    }
    for (int r = 0; r < N; ++r) {
      if (r == k) continue;
      const double f = A[r * N + k];
      for (int c = 0; c < N; ++c) {
        A[r * N + c] -= f * A[k * N + c];
        X[r * N + c] -= f * X[k * N + c];
      }
    }
  }
}

// Upper factor R of the Gram matrix of eq. GHYZ in xi on the monomials xi^1..xi^r
// (G = R^T R; the constant monomial has no derivative), row-major r x r
template <int r>
__device__ void gram_factor(double* R) {
  double G[r * r];
  for (int m = 1; m <= r; ++m)
    for (int n = 1; n <= r; ++n) {
      double s = 0.0;
      for (int l = 1; l <= (m < n ? m : n); ++l) {
        double fm = 1.0, fn = 1.0;
        for (int t = 0; t < l; ++t) {
          fm *= (m - t);
          fn *= (n - t);
        }
        s += fm * fn * imono(m + n - 2 * l, -0.5, 0.5);
      }
      G[(m - 1) * r + (n - 1)] = s;
    }
  for (int i = 0; i < r * r; ++i) R[i] = 0.0;
  for (int j = 0; j < r; ++j) {
    double d = G[j * r + j];
    for (int k = 0; k < j; ++k) d -= R[k * r + j] * R[k * r + j];
    const double rjj = sqrt(d);
    R[j * r + j] = rjj;
    for (int i = j + 1; i < r; ++i) {
      double v = G[j * r + i];
      for (int k = 0; k < j; ++k) v -= R[k * r + j] * R[k * r + i];
      R[j * r + i] = v / rjj;
    }
  }
}

// The polynomial of degree N - 1 fixed by N conditions (kind[q], cell j[q]): its monomial
// coefficients as linear maps of the conditions' data, C[m * N + q]
template <int N>
__device__ void poly_map(const int* kind, const int* j, const double* cc, const double* ww, double* C) {
  double A[N * N];
  for (int q = 0; q < N; ++q)
    for (int m = 0; m < N; ++m) A[q * N + m] = cond(kind[q], cc[j[q] + 1], ww[j[q] + 1], m);
  invert<N>(A, C);
}

// value of the polynomial at xi as a map of its data
template <int N>
__device__ void point_row(const double* C, double xi, double* row) {
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
    for (int m = N - 1; m >= 0; --m) s = s * xi + C[m * N + q];
    row[q] = s;
  }
}

// first moment over [-1/2, 1/2] as a map of the data
template <int N>
__device__ void moment_row(const double* C, double* row) {
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
    for (int m = 0; m < N; ++m) s += imono(m + 1, -0.5, 0.5) * C[m * N + q];
    row[q] = s;
  }
}

// indicator rows R C (rows 0..N-2, over the data) for the Gram factor of degree N - 1
template <int N>
__device__ void beta_rows(const double* C, double* rows) {
  constexpr int r = N - 1;
  double R[r * r];
  gram_factor<r>(R);
  for (int a = 0; a < r; ++a)
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
      for (int m = 1; m <= r; ++m) s += R[a * r + (m - 1)] * C[m * N + q];
      rows[a * N + q] = s;
    }
}

// one instance of n cells whose table columns start at column base of tables with stride
// columns per field
__global__ __launch_bounds__(256) void mesh1d_setup_kernel(const double* faces, int n, int bc,
                                                            double* tab, size_t stride, int base) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double dx = faces[i + 1] - faces[i];
  double dl, dr;   // neighbour sizes (periodic wrap; a mirrored ghost has the cell's size)
  if (bc == BC_PERIODIC) {
    dl = i > 0 ? faces[i] - faces[i - 1] : faces[n] - faces[n - 1];
    dr = i < n - 1 ? faces[i + 2] - faces[i + 1] : faces[1] - faces[0];
  } else {
    dl = i > 0 ? faces[i] - faces[i - 1] : dx;
    dr = i < n - 1 ? faces[i + 2] - faces[i + 1] : dx;
  }
  const double a = dl / dx, b = dr / dx;
  const double cc[3] = {-0.5 - 0.5 * a, 0.0, 0.5 + 0.5 * b}, ww[3] = {a, 1.0, b};
  auto put = [&](int k, const double* v, int len) {
    for (int q = 0; q < len; ++q) tab[(size_t)(k + q) * stride + base + i] = v[q];
  };
  const double one[1] = {dx};
  put(K_DX, one, 1);
  double row[6];
  {  // Step 1: quartic on the three cells' averages and the neighbours' first moments
    const int kind[5] = {0, 0, 0, 1, 1}, j[5] = {-1, 0, 1, -1, 1};
    double C[25], rows[20];
    poly_map<5>(kind, j, cc, ww, C);
    moment_row<5>(C, row);
    put(K_LQ0, row, 5);
    beta_rows<5>(C, rows);
    put(K_LB0, rows, 20);
  }
  {  // the linear q1, q2 and their slopes
    const int kind[2] = {0, 0}, jm[2] = {-1, 0}, jp[2] = {0, 1};
    double C[4];
    poly_map<2>(kind, jm, cc, ww, C);
    moment_row<2>(C, row);
    put(K_LQ1, row, 2);
    put(K_LB1, C + 2, 2);
    poly_map<2>(kind, jp, cc, ww, C);
    moment_row<2>(C, row);
    put(K_LQ2, row, 2);
    put(K_LB2, C + 2, 2);
  }
  {  // Step 2: quintic on the three cells' averages and first moments
    const int kind[6] = {0, 0, 0, 1, 1, 1}, j[6] = {-1, 0, 1, -1, 0, 1};
    double C[36], rows[30];
    poly_map<6>(kind, j, cc, ww, C);
    point_row<6>(C, -0.5, row);
    put(K_RL0, row, 6);
    point_row<6>(C, 0.5, row);
    put(K_RR0, row, 6);
    const double s5 = 0.223606797749978969640917366873127624;   // sqrt(5) / 10
    point_row<6>(C, -s5, row);
    put(K_RIM, row, 6);
    point_row<6>(C, s5, row);
    put(K_RIP, row, 6);
    beta_rows<6>(C, rows);
    put(K_RB0, rows, 30);
  }
  {  // the quadratics p1 (u_{-1}, u_0, v_0) and p2 (u_0, u_{+1}, v_0)
    const int kind[3] = {0, 0, 1}, jm[3] = {-1, 0, 0}, jp[3] = {0, 1, 0};
    double C[9], rows[6];
    poly_map<3>(kind, jm, cc, ww, C);
    point_row<3>(C, -0.5, row);
    put(K_RL1, row, 3);
    point_row<3>(C, 0.5, row);
    put(K_RR1, row, 3);
    beta_rows<3>(C, rows);
    put(K_RB1, rows, 6);
    poly_map<3>(kind, jp, cc, ww, C);
    point_row<3>(C, -0.5, row);
    put(K_RL2, row, 3);
    point_row<3>(C, 0.5, row);
    put(K_RR2, row, 3);
    beta_rows<3>(C, rows);
    put(K_RB2, rows, 6);
  }
}

}  // namespace mesh1d

}  // namespace hw

template <int EQ, int T>
static void launch1d(int persistent, int grid, const hw::Stage1D* P, hipStream_t s) {
  if (persistent) hipLaunchKernelGGL((hw::stage1d_persistent<EQ, T>), dim3(grid), dim3(T), 0, s, *P);
  else hipLaunchKernelGGL((hw::stage1d_kernel<EQ, T, false>), dim3(P->nitems), dim3(T), 0, s, *P);
}

template <int EQ>
static hipError_t launch1d_tile(int persistent, int grid, int tile, const hw::Stage1D* P, hipStream_t s) {
  switch (tile) {
    case 64: launch1d<EQ, 64>(persistent, grid, P, s); break;
    case 128: launch1d<EQ, 128>(persistent, grid, P, s); break;
    case 256: launch1d<EQ, 256>(persistent, grid, P, s); break;
    case 512: launch1d<EQ, 512>(persistent, grid, P, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_stage1d(int eq, int persistent, int grid, int tile,
                                        const hw::Stage1D* P, hipStream_t s) {
  if (P->nu) {
    // cells of different sizes: one instance, 256-cell tiles, one workgroup per tile
    dim3 g(P->nitems), b(256);
    if (eq == hw::EQ_EULER) hipLaunchKernelGGL((hw::stage1d_kernel<hw::EQ_EULER, 256, true>), g, b, 0, s, *P);
    else if (eq == hw::EQ_BURGERS) hipLaunchKernelGGL((hw::stage1d_kernel<hw::EQ_BURGERS, 256, true>), g, b, 0, s, *P);
    else if (eq == hw::EQ_ADV) hipLaunchKernelGGL((hw::stage1d_kernel<hw::EQ_ADV, 256, true>), g, b, 0, s, *P);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (eq == hw::EQ_EULER) return launch1d_tile<hw::EQ_EULER>(persistent, grid, tile, P, s);
  if (eq == hw::EQ_BURGERS) return launch1d_tile<hw::EQ_BURGERS>(persistent, grid, tile, P, s);
  if (eq == hw::EQ_ADV) return launch1d_tile<hw::EQ_ADV>(persistent, grid, tile, P, s);
  return hipErrorInvalidValue;
}

extern "C" hipError_t hw_launch_alpha1d(int eq, const double* U, const int* off, int ninst,
                                        int total, int maxn, double gam, double adv,
                                        unsigned long long* alpha_out, hipStream_t s) {
  int bx = (maxn + 255) / 256;
  if (bx > 64) bx = 64;
  dim3 g(bx, ninst), b(256);
  if (eq == hw::EQ_EULER)
    hipLaunchKernelGGL(hw::alpha1d_kernel<hw::EQ_EULER>, g, b, 0, s, U, off, total, gam, adv, alpha_out);
  else if (eq == hw::EQ_BURGERS)
    hipLaunchKernelGGL(hw::alpha1d_kernel<hw::EQ_BURGERS>, g, b, 0, s, U, off, total, gam, adv, alpha_out);
  else
    hipLaunchKernelGGL(hw::alpha1d_kernel<hw::EQ_ADV>, g, b, 0, s, U, off, total, gam, adv, alpha_out);
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_mesh1d_setup(const double* faces, int n, int bc, double* tab,
                                             hipStream_t s) {
  hipLaunchKernelGGL(hw::mesh1d::mesh1d_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                     faces, n, bc, tab, (size_t)n, 0);
  return hipGetLastError();
}

extern "C" hipError_t hw_launch_mesh1d_setup_batch(const double* faces, const int* off, int ninst,
                                                   int bc, double* tab, int total, hipStream_t s) {
  for (int b = 0; b < ninst; ++b) {
    const int n = off[b + 1] - off[b];
    // instance b's faces follow those of the instances before it (n + 1 each)
    hipLaunchKernelGGL(hw::mesh1d::mesh1d_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                       faces + off[b] + b, n, bc, tab, (size_t)total, off[b]);
  }
  return hipGetLastError();
}

#!/usr/bin/env python3
"""Generate hw_coeffs2d.h: the two-dimensional reconstruction operators of Step 5.1
(Zhao & Qiu, arXiv 2002.08816, Section 2.2) as straight-line device code.

Derivation (exact, sympy), in reference coordinates (xi, eta) in [-1/2, 1/2]^2 of the
target cell, neighbours at integer offsets (labels 1..9 of Figure 1):

* p0 (quartic, 15 monomials): the nine averages and the two first moments of the target
  cell are met exactly; the first moments of the four edge neighbours (labels 2, 4, 6, 8)
  in the unweighted least-squares sense.  Solved in null-space form: a particular
  solution of the exact rows plus the null-space component minimising the residual.
* p1..p4 (quadratics, 6 monomials): the averages of the 2x2 sub-stencils of Figure 2 and
  the two first moments of the target cell, interpolated.
* smoothness indicators (eq. 2dGHYZ, square cells): Gram matrices of the derivative
  integrals over the target cell, each multi-index counted once.

Emitted code
* lin2d_inner / lin2d_xedges_ng<NG> / lin2d_yedges_ng<NG>: the linear path (Steps 5.2
  and 5.3) for one field: values of p0 at the 3 x 3 interior Gauss points, at the Gauss
  points of the left and right edges, and of the bottom and top edges.  The stencil data are folded into the four reflection-parity classes of the
  3x3 stencil (even/odd under xi -> -xi and under eta -> -eta); since p0 commutes with
  both reflections, each parity part of a point value depends only on the inputs of the
  same class, and the four mirror images of a point follow by a butterfly.  This cuts
  the multiply count per field to about a quarter of the dense map.
* p0_coeffs / pq_coeffs<n>: monomial coefficients of p0 and p_n, for the HWENO path.
* beta_p0 / beta_pq: the smoothness indicators as sparse quadratic forms.
* edge monomial tables for evaluating the candidates at the edge Gauss points.

Input order of the 19 stencil values ("in"):
  0..8   averages of labels 1..9
  9..13  x first moments of labels 2, 4, 5, 6, 8
  14..18 y first moments of labels 2, 4, 5, 6, 8
Edge point order: left (-1/2, e_k), right (1/2, e_k), bottom (e_k, -1/2), top (e_k, 1/2)
with e_k the ascending Gauss nodes; interior (g_k, g_l) at index 3 l + k (3-point Gauss).

Run: python gen_coeffs2d.py > hw_coeffs2d.h
"""
import sys

import sympy as sp

HALF = sp.Rational(1, 2)


def cell_int(m, j):
    x = sp.Symbol("x")
    return sp.integrate(x ** m, (x, j - HALF, j + HALF))


def cell_int_w(m, j):
    x = sp.Symbol("x")
    return sp.integrate(x ** m * (x - j), (x, j - HALF, j + HALF))


def offset(label):
    return (label - 1) % 3 - 1, (label - 1) // 3 - 1


def monos(r):
    return [(p, t - p) for t in range(r + 1) for p in range(t, -1, -1)]


CROSS = (2, 4, 5, 6, 8)
IN_NAMES = ([f"u{k}" for k in range(1, 10)] + [f"v{k}" for k in CROSS] + [f"w{k}" for k in CROSS])


def in_index(kind, label):
    if kind == "u":
        return label - 1
    base = 9 if kind == "v" else 14
    return base + CROSS.index(label)


def moment_row(kind, label, mons):
    a, b = offset(label)
    row = []
    for p, q in mons:
        if kind == "u":
            row.append(cell_int(p, a) * cell_int(q, b))
        elif kind == "v":
            row.append(cell_int_w(p, a) * cell_int(q, b))
        else:
            row.append(cell_int(p, a) * cell_int_w(q, b))
    return row


def derive_p0():
    mons = monos(4)
    ex = [("u", k) for k in range(1, 10)] + [("v", 5), ("w", 5)]
    ls = [(kd, k) for k in (2, 4, 6, 8) for kd in ("v", "w")]
    E = sp.Matrix([moment_row(kd, k, mons) for kd, k in ex])
    B = sp.Matrix([moment_row(kd, k, mons) for kd, k in ls])
    # selector matrices from the 19 inputs
    SE = sp.zeros(len(ex), 19)
    for i, (kd, k) in enumerate(ex):
        SE[i, in_index(kd, k)] = 1
    SB = sp.zeros(len(ls), 19)
    for i, (kd, k) in enumerate(ls):
        SB[i, in_index(kd, k)] = 1
    # particular solution: minimum-norm-free choice via pivot columns of E
    N = E.nullspace()
    assert len(N) == 4
    N = sp.Matrix.hstack(*N)
    Ep = E.pinv()
    # c = Ep SE d + N z ;  minimise |B c - SB d|^2 over z
    BN = B * N
    z_map = -(BN.T * BN).inv() * BN.T * (B * Ep * SE - SB)
    C = Ep * SE + N * z_map
    C = C.applyfunc(sp.simplify)
    assert (E * C - SE).applyfunc(sp.simplify) == sp.zeros(len(ex), 19)
    return mons, C


SUB = {1: (1, 2, 4, 5), 2: (2, 3, 5, 6), 3: (4, 5, 7, 8), 4: (5, 6, 8, 9)}


def derive_pq(n):
    mons = monos(2)
    conds = [("u", k) for k in SUB[n]] + [("v", 5), ("w", 5)]
    A = sp.Matrix([moment_row(kd, k, mons) for kd, k in conds])
    S = sp.zeros(6, 19)
    for i, (kd, k) in enumerate(conds):
        S[i, in_index(kd, k)] = 1
    return mons, A.inv() * S


def int_sym(a):
    """Integral of x^a over [-1/2, 1/2]."""
    return sp.Integer(0) if a % 2 else 2 * HALF ** (a + 1) / (a + 1)


def dmono(p, l):
    """(coefficient, exponent) of d^l/dx^l x^p."""
    if l > p:
        return sp.Integer(0), 0
    c = sp.Integer(1)
    for t in range(l):
        c *= (p - t)
    return c, p - l


def gram(mons, r):
    G = sp.zeros(len(mons), len(mons))
    for L in range(1, r + 1):
        for l1 in range(L + 1):
            l2 = L - l1
            for s, (p, q) in enumerate(mons):
                cp, ep = dmono(p, l1)
                cq, eq = dmono(q, l2)
                if cp == 0 or cq == 0:
                    continue
                for t, (p2, q2) in enumerate(mons):
                    cp2, ep2 = dmono(p2, l1)
                    cq2, eq2 = dmono(q2, l2)
                    if cp2 == 0 or cq2 == 0:
                        continue
                    G[s, t] += cp * cq * cp2 * cq2 * int_sym(ep + ep2) * int_sym(eq + eq2)
    return G


def gauss_nodes(ng):
    if ng == 2:
        return [-sp.sqrt(3) / 6, sp.sqrt(3) / 6]
    return [-sp.sqrt(15) / 10, sp.Integer(0), sp.sqrt(15) / 10]


def cnum(v):
    f = float(sp.N(v, 40))
    return repr(f)


def emit_sum(terms, indent="  "):
    """terms: list of (coef, expr_string); returns an expression using fma chains."""
    terms = [(c, e) for c, e in terms if c != 0]
    if not terms:
        return "0.0"
    c0, e0 = terms[0]
    acc = e0 if c0 == 1 else f"{cnum(c0)} * {e0}"
    for c, e in terms[1:]:
        acc = f"fma({cnum(c)}, {e}, {acc})"
    return acc


# ------------------------------------------------------------------ parity folding
# class -> list of (name, {input_index: sign})
def folded_inputs():
    u = lambda k: in_index("u", k)
    v = lambda k: in_index("v", k)
    w = lambda k: in_index("w", k)
    return {
        "ee": [{u(5): 1}, {u(4): 1, u(6): 1}, {u(2): 1, u(8): 1}, {u(1): 1, u(3): 1, u(7): 1, u(9): 1},
               {v(6): 1, v(4): -1}, {w(8): 1, w(2): -1}],
        "oe": [{u(6): 1, u(4): -1}, {u(3): 1, u(9): 1, u(1): -1, u(7): -1}, {v(5): 1},
               {v(4): 1, v(6): 1}, {v(2): 1, v(8): 1}],
        "eo": [{u(8): 1, u(2): -1}, {u(7): 1, u(9): 1, u(1): -1, u(3): -1}, {w(5): 1},
               {w(2): 1, w(8): 1}, {w(4): 1, w(6): 1}],
        "oo": [{u(1): 1, u(9): 1, u(3): -1, u(7): -1}, {v(8): 1, v(2): -1}, {w(6): 1, w(4): -1}],
    }


def parity_part_rows(row, cls_inputs):
    """Express the parity part of the linear functional `row` (over the 19 inputs) in
    terms of the folded inputs of one class.  The folded inputs of a class are mutually
    orthogonal sign patterns over disjoint supports, so the coefficient of folded input f
    is row . f / |f|^2."""
    out = []
    for f in cls_inputs:
        num = sum(row[i] * s for i, s in f.items())
        den = sum(s * s for s in f.values())
        out.append(sp.simplify(num / den))
    return out


def main():
    mons4, C0 = derive_p0()
    pq = {n: derive_pq(n) for n in (1, 2, 3, 4)}
    mons2 = pq[1][0]
    G4 = gram(mons4, 4)
    G2 = gram(mons2, 2)
    classes = folded_inputs()
    cls_sign = {"ee": (1, 1), "oe": (-1, 1), "eo": (1, -1), "oo": (-1, -1)}

    def value_row(C, mons, x, y):
        return [sp.simplify(sum(C[s, k] * x ** p * y ** q for s, (p, q) in enumerate(mons)))
                for k in range(19)]

    out = []
    w = out.append
    w("// Generated by gen_coeffs2d.py -- do not edit.")
    w("// Two-dimensional reconstruction operators of Step 5.1 (Section 2.2): the least-squares")
    w("// quartic p0 (Figure 1 stencil), the quadratics p1..p4 (Figure 2 sub-stencils) and the")
    w("// smoothness indicators of eq. 2dGHYZ for square cells.")
    w("#pragma once")
    w("namespace hw2 {")
    w("")
    w("// ---------------------------------------------------------------- linear path")
    w("// Point values of p0 for one field: reflection-parity folding of the 19 inputs,")
    w("// then a butterfly per orbit of mirror-image points.")
    def emit_points(fname, pts_and_targets):
        """One straight-line function: fold the inputs, evaluate the parity parts at the
        representative points, and assemble the requested point values."""
        w(f"__device__ __forceinline__ void {fname} {{")
        for cls, fl in classes.items():
            for i, f in enumerate(fl):
                terms = []
                for idx, sg in f.items():
                    terms.append(("+" if sg > 0 else "-") + f"in[{idx}]")
                expr = " ".join(terms).lstrip("+").strip()
                w(f"  const double {cls}{i} = {expr};")
        reps.clear()
        for target, (x, y) in pts_and_targets:
            w(f"  {target} = {point(x, y)};")
        w("}")
        w("")

    reps = {}

    def part(cls, x, y):
        key = (cls, x, y)
        if key in reps:
            return reps[key]
        row = value_row(C0, mons4, x, y)
        coefs = parity_part_rows(row, classes[cls])
        name = f"P{cls}_{len(reps)}"
        w(f"  const double {name} = {emit_sum([(c, f'{cls}{i}') for i, c in enumerate(coefs)])};")
        reps[key] = name
        return name

    def point(x, y):
        """expression for p0 at (x, y) from the parity parts at (|x|, |y|)."""
        ax, ay = abs(x), abs(y)
        sx = -1 if x < 0 else 1
        sy = -1 if y < 0 else 1
        terms = []
        for cls, (px, py) in cls_sign.items():
            if (px == -1 and ax == 0) or (py == -1 and ay == 0):
                continue   # odd part vanishes on the mirror line
            sgn = (sx if px == -1 else 1) * (sy if py == -1 else 1)
            terms.append((sgn, part(cls, ax, ay)))
        # self-check: the parity parts add up to the dense row of p0 at (x, y)
        dense = value_row(C0, mons4, x, y)
        back = [sp.Integer(0)] * 19
        for cls, (px, py) in cls_sign.items():
            if (px == -1 and ax == 0) or (py == -1 and ay == 0):
                continue
            sgn = (sx if px == -1 else 1) * (sy if py == -1 else 1)
            coefs = parity_part_rows(value_row(C0, mons4, ax, ay), classes[cls])
            for f, c in zip(classes[cls], coefs):
                for idx, sg in f.items():
                    back[idx] += sgn * c * sg
        assert all(sp.simplify(a - b) == 0 for a, b in zip(dense, back)), (x, y)
        expr = ""
        for sgn, nm in terms:
            expr += (" + " if sgn > 0 else " - ") + nm
        expr = expr.strip()
        if expr.startswith("+ "):
            expr = expr[2:]
        elif expr.startswith("- "):
            expr = "-" + expr[2:]
        return expr

    inner_nodes = gauss_nodes(3)
    emit_points("lin2d_inner(const double* in, double* inner)",
                [(f"inner[{3 * l + k}]", (a, b)) for l, b in enumerate(inner_nodes)
                 for k, a in enumerate(inner_nodes)])
    for ng in (2, 3):
        nodes = gauss_nodes(ng)
        emit_points(f"lin2d_xedges_ng{ng}(const double* in, double* xl, double* xr)",
                    [(f"xl[{k}]", (-HALF, e)) for k, e in enumerate(nodes)]
                    + [(f"xr[{k}]", (HALF, e)) for k, e in enumerate(nodes)])
        emit_points(f"lin2d_yedges_ng{ng}(const double* in, double* yb, double* yt)",
                    [(f"yb[{k}]", (e, -HALF)) for k, e in enumerate(nodes)]
                    + [(f"yt[{k}]", (e, HALF)) for k, e in enumerate(nodes)])

    # ---------------------------------------------------------------- HWENO path
    w("// ---------------------------------------------------------------- HWENO path")
    w("// Monomial order (p, q) for xi^p eta^q: by total degree, then descending p.")
    w("__device__ __forceinline__ void p0_coeffs(const double* in, double* c) {")
    for s in range(15):
        w(f"  c[{s}] = {emit_sum([(C0[s, k], f'in[{k}]') for k in range(19)])};")
    w("}")
    for n in (1, 2, 3, 4):
        mons, C = pq[n]
        w(f"__device__ __forceinline__ void p{n}_coeffs(const double* in, double* c) {{")
        for s in range(6):
            w(f"  c[{s}] = {emit_sum([(C[s, k], f'in[{k}]') for k in range(19)])};")
        w("}")

    def emit_quad(G, n, name):
        w(f"__device__ __forceinline__ double {name}(const double* c) {{")
        w("  double b = 0.0;")
        for s in range(n):
            terms = []
            if G[s, s] != 0:
                terms.append((G[s, s], f"c[{s}]"))
            for t in range(s + 1, n):
                if G[s, t] != 0:
                    terms.append((2 * G[s, t], f"c[{t}]"))
            if terms:
                w(f"  b = fma(c[{s}], {emit_sum(terms)}, b);")
        w("  return b;")
        w("}")

    emit_quad(G4, 15, "beta_p0")
    emit_quad(G2, 6, "beta_pq")
    for ng in (2, 3):
        nodes = gauss_nodes(ng)
        pts = ([(-HALF, e) for e in nodes] + [(HALF, e) for e in nodes]
               + [(e, -HALF) for e in nodes] + [(e, HALF) for e in nodes])
        w(f"// value of a quartic (15 coefficients) or quadratic (first 6) at edge point i")
        w(f"__device__ __forceinline__ double edge_quartic_ng{ng}(const double* c, int i) {{")
        w("  switch (i) {")
        for i, (x, y) in enumerate(pts):
            w(f"  case {i}: return {emit_sum([(x ** p * y ** q, f'c[{s}]') for s, (p, q) in enumerate(mons4)])};")
        w("  }")
        w("  return 0.0;")
        w("}")
        w(f"__device__ __forceinline__ double edge_quad_ng{ng}(const double* c, int i) {{")
        w("  switch (i) {")
        for i, (x, y) in enumerate(pts):
            w(f"  case {i}: return {emit_sum([(x ** p * y ** q, f'c[{s}]') for s, (p, q) in enumerate(mons2)])};")
        w("  }")
        w("  return 0.0;")
        w("}")
    # ---------------------------------------------------------------- adjoint pieces
    w("// ---------------------------------------------------------------- adjoint path")
    w("// Transposes (accumulating into db[19]) of the linear point maps, of the candidate")
    w("// coefficient maps and of the edge evaluations; gradients of the indicators.")

    def emit_transpose(fname, points):
        """db[j] += sum_k R[k][j] * ub[k] for the dense rows R of p0 at the points."""
        rows = [value_row(C0, mons4, x, y) for (x, y) in points]
        w(f"__device__ __forceinline__ void {fname} {{")
        for j in range(19):
            terms = [(rows[k][j], f"ub[{k}]") for k in range(len(points))]
            terms = [(c, e) for c, e in terms if c != 0]
            if not terms:
                continue
            acc = f"db[{j}]"
            for c, e in terms:
                acc = f"fma({cnum(c)}, {e}, {acc})"
            w(f"  db[{j}] = {acc};")
        w("}")
        w("")

    emit_transpose("lin2d_inner_T(const double* ub, double* db)",
                   [(a, b) for b in inner_nodes for a in inner_nodes])
    for ng in (2, 3):
        nodes = gauss_nodes(ng)
        emit_transpose(f"lin2d_xedges_ng{ng}_T(const double* ub, double* db)",
                       [(-HALF, e) for e in nodes] + [(HALF, e) for e in nodes])
        emit_transpose(f"lin2d_yedges_ng{ng}_T(const double* ub, double* db)",
                       [(e, -HALF) for e in nodes] + [(e, HALF) for e in nodes])

    def emit_coef_T(fname, C, n):
        w(f"__device__ __forceinline__ void {fname}(const double* cb, double* db) {{")
        for j in range(19):
            terms = [(C[t, j], f"cb[{t}]") for t in range(n) if C[t, j] != 0]
            if not terms:
                continue
            acc = f"db[{j}]"
            for c, e in terms:
                acc = f"fma({cnum(c)}, {e}, {acc})"
            w(f"  db[{j}] = {acc};")
        w("}")

    emit_coef_T("p0_coeffs_T", C0, 15)
    for n in (1, 2, 3, 4):
        emit_coef_T(f"p{n}_coeffs_T", pq[n][1], 6)

    def emit_grad(G, n, name):
        w(f"// gradient 2 G c of the quadratic form c^T G c")
        w(f"__device__ __forceinline__ void {name}(const double* c, double* g) {{")
        for t in range(n):
            terms = [(2 * G[t, u], f"c[{u}]") for u in range(n) if G[t, u] != 0]
            w(f"  g[{t}] = {emit_sum(terms)};")
        w("}")

    emit_grad(G4, 15, "beta_p0_grad")
    emit_grad(G2, 6, "beta_pq_grad")
    for ng in (2, 3):
        nodes = gauss_nodes(ng)
        pts = ([(-HALF, e) for e in nodes] + [(HALF, e) for e in nodes]
               + [(e, -HALF) for e in nodes] + [(e, HALF) for e in nodes])
        w(f"// transposes of edge_quartic / edge_quad: cb[s] += mono_s(point i) * qb")
        w(f"__device__ __forceinline__ void edge_quartic_ng{ng}_T(double qb, int i, double* cb) {{")
        w("  switch (i) {")
        for i, (x, y) in enumerate(pts):
            body = " ".join(f"cb[{t}] = fma({cnum(x ** p * y ** q)}, qb, cb[{t}]);"
                            for t, (p, q) in enumerate(mons4) if x ** p * y ** q != 0)
            w(f"  case {i}: {body} break;")
        w("  }")
        w("}")
        w(f"__device__ __forceinline__ void edge_quad_ng{ng}_T(double qb, int i, double* cb) {{")
        w("  switch (i) {")
        for i, (x, y) in enumerate(pts):
            body = " ".join(f"cb[{t}] = fma({cnum(x ** p * y ** q)}, qb, cb[{t}]);"
                            for t, (p, q) in enumerate(mons2) if x ** p * y ** q != 0)
            w(f"  case {i}: {body} break;")
        w("  }")
        w("}")
    w("")
    w("}  // namespace hw2")
    sys.stdout.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()

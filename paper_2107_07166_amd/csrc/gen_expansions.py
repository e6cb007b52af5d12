"""Generates expansions_gen.h: straight-line Cartesian-tensor FMM operators.

The GPU kernels need, for every expansion order P = 1..8, fully unrolled code
for (notation of Korobkin et al., arXiv:2107.07166, Sec. 2):

* the derivative tensors of the softened kernels at R (the D tensors of the
  paper, generalised to any order and to softening),
    phi(r) = -(|r|^2 + eps^2)^(-1/2),  g(r) = (|r|^2 + eps^2)^(-3/2) = F_1;
  with F_n(s) = 2^n d^n/ds^n [-s^(-1/2)], s = |r|^2 + eps^2, the radial
  functions satisfy F_0 = -s^(-1/2), F_{n+1} = -(2n+1) F_n / s, and
  d_r F_n = r F_{n+1}.  The tensors A^(n)_k = d^k F_n then obey
      A^(n)_{k+e_d} = R_d A^(n+1)_k + k_d A^(n+1)_{k-e_d},
  so phi-derivatives are layer n = 0 and g-derivatives are layer n = 1;
* the standard M2L contraction (the Taylor series of Eq. taylor summed over
  the source node, as in Eqs. potential / g_acc_BtoA):
      L_j += sum_{|i| <= P-|j|} D_{i+j} W_i,  W_i = (-1)^|i| M_i / i!;
* the conserving M2L contraction (realigned force, Eq. realign, with the
  projection scalar kept to degree P-1): the far field of B at x is
      a_e(x) = -(R_e + x_e) P(x) + Q_e(x),
      P_j  = sum_{|i| <= P-1-|j|} G_{i+j} W_i,
      Q_ej = sum_{|i| <= P-1-|j|} (-1)^|i| G_{i+j} M_{i+e} / i!
           = -sum (i_e + 1) G_{i+j} W_{i+e};
  the -R_e P term is folded in per pair, so the node accumulates P and
  Q'_e = Q_e - R_e P;
* the exact polynomial shift of local expansions (L2L) and the evaluation at
  a particle (L2P).

Multi-indices k = (kx, ky, kz) are stored in graded order: all |k| = n after
all |k| < n, and within a degree by a = ky + kz ascending, then kz ascending:
    idx(k) = n(n+1)(n+2)/6 + a(a+1)/2 + kz.
Dipole moments about the centre of mass vanish, so W_i with |i| = 1 is never
read.

Run:  python gen_expansions.py  (writes expansions_gen.h next to this file).
"""

import os
import sys

PMAX = 8


def c_le(n):
    return (n + 1) * (n + 2) * (n + 3) // 6 if n >= 0 else 0


def idx(k):
    kx, ky, kz = k
    n = kx + ky + kz
    a = ky + kz
    return c_le(n - 1) + a * (a + 1) // 2 + kz


def multi(n):
    out = []
    for a in range(n + 1):
        for kz in range(a + 1):
            out.append((n - a, a - kz, kz))
    return out


def all_upto(p):
    out = []
    for n in range(p + 1):
        out.extend(multi(n))
    return out


def add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
AX = "xyz"


def fmt(c):
    """A floating constant valid for both float and double (cast to T)."""
    if float(c).is_integer():
        return f"T({int(c)})"
    return f"T({c!r})"


def gen_layers(P, stop):
    """Code computing A^(n)_k for n = P..stop, |k| <= P-n.  Returns lines and
    the variable name of A^(stop)_k."""
    lines = []
    name = {}
    for n in range(P, stop - 1, -1):
        for k in all_upto(P - n):
            v = f"a{n}_{idx(k)}"
            name[(n, k)] = v
            if sum(k) == 0:
                lines.append(f"const T {v} = F[{n}];")
                continue
            d = 0 if k[0] else (1 if k[1] else 2)
            k1 = list(k)
            k1[d] -= 1
            k1 = tuple(k1)
            r = "xyz"[d]
            term = f"R{r} * {name[(n + 1, k1)]}"
            if k[d] >= 2:
                k2 = list(k1)
                k2[d] -= 1
                k2 = tuple(k2)
                coef = k[d] - 1
                if coef == 1:
                    term = f"fma(R{r}, {name[(n + 1, k1)]}, {name[(n + 1, k2)]})"
                else:
                    term = f"fma(R{r}, {name[(n + 1, k1)]}, {fmt(coef)} * {name[(n + 1, k2)]})"
            lines.append(f"const T {v} = {term};")
    return lines, name


def gen_struct(P):
    NC = c_le(P)
    NC1 = c_le(P - 1)
    out = [f"template <> struct Expansion<{P}> {{",
           f"  static constexpr int P = {P};",
           f"  static constexpr int NC = {NC};",
           f"  static constexpr int NC1 = {NC1};"]

    # phi derivatives (layer 0), |k| <= P
    lines, name = gen_layers(P, 0)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void phi_derivs(T Rx, T Ry, T Rz, const T* F, T* D) {")
    out += ["    " + s for s in lines]
    for k in all_upto(P):
        out.append(f"    D[{idx(k)}] = {name[(0, k)]};")
    out.append("  }")

    # g derivatives (layer 1), |k| <= P-1
    lines, name = gen_layers(P, 1)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void g_derivs(T Rx, T Ry, T Rz, const T* F, T* G) {")
    out += ["    " + s for s in lines]
    for k in all_upto(P - 1):
        out.append(f"    G[{idx(k)}] = {name[(1, k)]};")
    out.append("  }")

    # standard M2L: L_j += sum_i D_{i+j} W_i, 1 <= |j| <= P (|j| = 0 only with WITH_POT)
    out.append("  template <typename T, bool WITH_POT>")
    out.append("  __device__ __forceinline__ static void m2l_std(const T* D, const T* W, T* L) {")
    for j in all_upto(P):
        if sum(j) == 0:
            out.append("    if (WITH_POT) {")
            pre = "      "
        else:
            pre = "    "
        terms = [(idx(add(i, j)), idx(i)) for i in all_upto(P - sum(j)) if sum(i) != 1]
        expr = f"L[{idx(j)}]"
        for di, wi in terms:
            expr = f"fma(D[{di}], W[{wi}], {expr})"
        out.append(f"{pre}L[{idx(j)}] = {expr};")
        if sum(j) == 0:
            out.append("    }")
    out.append("  }")

    # conserving M2L: P_j and Q'_ej = Q_ej - R_e P_j(pair)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void m2l_cons(const T* G, const T* W, T Rx, T Ry, T Rz,"
               " T* Pa, T* Qa) {")
    for j in all_upto(P - 1):
        terms = [(idx(add(i, j)), idx(i)) for i in all_upto(P - 1 - sum(j)) if sum(i) != 1]
        expr = None
        for gi, wi in terms:
            expr = f"G[{gi}] * W[{wi}]" if expr is None else f"fma(G[{gi}], W[{wi}], {expr})"
        if expr is None:
            expr = "T(0)"
        out.append(f"    {{ const T pj = {expr};")
        out.append(f"      Pa[{idx(j)}] += pj;")
        for e in range(3):
            qterms = []
            for i in all_upto(P - 1 - sum(j)):
                if sum(i) == 0:
                    continue  # W_e (dipole) vanishes
                qterms.append((idx(add(i, j)), idx(add(i, E[e])), i[e] + 1))
            expr_q = f"-R{AX[e]} * pj"
            qa = f"Qa[{e * NC1 + idx(j)}]"
            # Q'_ej += sum -(i_e+1) G W  - R_e pj
            acc = None
            for gi, wi, c in qterms:
                t = f"G[{gi}] * W[{wi}]" if c == 1 else f"{fmt(c)} * (G[{gi}] * W[{wi}])"
                acc = t if acc is None else f"{acc} + {t}"
            if acc is None:
                out.append(f"      {qa} = fma(-R{AX[e]}, pj, {qa});")
            else:
                out.append(f"      {qa} = {qa} - (({acc}) + R{AX[e]} * pj);")
        out.append("    }")
    out.append("  }")

    # conserving M2L one polynomial at a time (for orders whose four
    # accumulator sets do not fit the registers together):
    #   cons_p:    Pa_j  += sum_{|i| <= P-1-|j|, |i| != 1} G_{i+j} W_i
    #   cons_q<E>: Qa_j  -= sum_{|i| <= P-1-|j|} G_{i+j} V_i,
    #              V_i = (i_E + 1) W_{i+E} [|i| >= 1] + R_E W_i [|i| != 1],
    # the same terms as m2l_cons (Q_Ej - R_E p_j) grouped per source moment.
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void cons_p(const T* G, const T* W, T* Pa) {")
    for j in all_upto(P - 1):
        terms = [(idx(add(i, j)), idx(i)) for i in all_upto(P - 1 - sum(j)) if sum(i) != 1]
        expr = f"Pa[{idx(j)}]"
        for gi, wi in terms:
            expr = f"fma(G[{gi}], W[{wi}], {expr})"
        out.append(f"    Pa[{idx(j)}] = {expr};")
    out.append("  }")
    for e in range(3):
        out.append("  template <typename T>")
        out.append(f"  __device__ __forceinline__ static void cons_q{AX[e]}(const T* G, const T* W, T R{AX[e]}, T* Qa) {{")
        for i in all_upto(P - 1):
            parts = []
            if sum(i) >= 1:
                c = i[e] + 1
                wi = idx(add(i, E[e]))
                parts.append(f"W[{wi}]" if c == 1 else f"{fmt(c)} * W[{wi}]")
            if sum(i) != 1:
                parts.append(f"R{AX[e]} * W[{idx(i)}]")
            if len(parts) == 2:
                if parts[0].startswith("W["):
                    v = f"fma(R{AX[e]}, W[{idx(i)}], {parts[0]})"
                else:
                    v = f"fma(R{AX[e]}, W[{idx(i)}], {parts[0]})"
            else:
                v = parts[0]
            out.append(f"    {{ const T v = {v};")
            for j in all_upto(P - 1 - sum(i)):
                out.append(f"      Qa[{idx(j)}] = fma(-G[{idx(add(i, j))}], v, Qa[{idx(j)}]);")
            out.append("    }")
        out.append("  }")

    # monomials x^j / j! for |j| <= Q (into Mo)
    def mono_lines(Q, var="Mo", dx="dx", dy="dy", dz="dz"):
        ls = [f"{var}[0] = T(1);"]
        for k in all_upto(Q)[1:]:
            d = 0 if k[0] else (1 if k[1] else 2)
            k1 = list(k)
            k1[d] -= 1
            dv = (dx, dy, dz)[d]
            if k[d] == 1:
                ls.append(f"{var}[{idx(k)}] = {var}[{idx(tuple(k1))}] * {dv};")
            else:
                ls.append(f"{var}[{idx(k)}] = {var}[{idx(tuple(k1))}] * ({dv} * {fmt(1.0 / k[d])});")
        return ls

    # L2L (standard): Ld_j += sum_{|i| <= P-|j|} Ls_{i+j} d^i/i!
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void shift_std(const T* Ls, T dx, T dy, T dz, T* Ld) {")
    out.append(f"    T Mo[{NC}];")
    out += ["    " + s for s in mono_lines(P)]
    for j in all_upto(P):
        terms = [(idx(add(i, j)), idx(i)) for i in all_upto(P - sum(j))]
        expr = f"Ld[{idx(j)}]"
        for li, mi in terms:
            expr = f"fma(Ls[{li}], Mo[{mi}], {expr})"
        out.append(f"    Ld[{idx(j)}] = {expr};")
    out.append("  }")

    # L2L (conserving): P' = shift(P); Q'_e = shift(Q_e) - d_e shift(P)   (degree P-1)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void shift_cons(const T* Ps, const T* Qs, T dx, T dy, T dz,"
               " T* Pd, T* Qd) {")
    out.append(f"    T Mo[{max(NC1, 1)}];")
    out += ["    " + s for s in mono_lines(P - 1)]
    for j in all_upto(P - 1):
        terms = [(idx(add(i, j)), idx(i)) for i in all_upto(P - 1 - sum(j))]
        sp = None
        for li, mi in terms:
            sp = f"Ps[{li}] * Mo[{mi}]" if sp is None else f"fma(Ps[{li}], Mo[{mi}], {sp})"
        out.append(f"    {{ const T sp = {sp};")
        out.append(f"      Pd[{idx(j)}] += sp;")
        for e in range(3):
            sq = None
            for li, mi in terms:
                sq = f"Qs[{e * NC1 + li}] * Mo[{mi}]" if sq is None else f"fma(Qs[{e * NC1 + li}], Mo[{mi}], {sq})"
            d = ("dx", "dy", "dz")[e]
            out.append(f"      Qd[{e * NC1 + idx(j)}] += fma(-{d}, sp, {sq});")
        out.append("    }")
    out.append("  }")

    # L2P (standard): a_e = -sum_{|j| <= P-1} L_{j+e} x^j/j!
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void l2p_std(const T* L, T dx, T dy, T dz, T* a) {")
    out.append(f"    T Mo[{max(NC1, 1)}];")
    out += ["    " + s for s in mono_lines(P - 1)]
    for e in range(3):
        expr = None
        for j in all_upto(P - 1):
            t = (idx(add(j, E[e])), idx(j))
            expr = f"L[{t[0]}] * Mo[{t[1]}]" if expr is None else f"fma(L[{t[0]}], Mo[{t[1]}], {expr})"
        out.append(f"    a[{e}] = -({expr});")
    out.append("  }")

    # L2P potential (standard locals, L_0 included): phi = sum_{|j| <= P} L_j x^j/j!
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static T l2p_pot(const T* L, T dx, T dy, T dz) {")
    out.append(f"    T Mo[{NC}];")
    out += ["    " + s for s in mono_lines(P)]
    expr = None
    for j in all_upto(P):
        expr = f"L[{idx(j)}] * Mo[{idx(j)}]" if expr is None else f"fma(L[{idx(j)}], Mo[{idx(j)}], {expr})"
    out.append(f"    return {expr};")
    out.append("  }")

    # L2P (conserving): a_e = -x_e P(x) + Q'_e(x)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void l2p_cons(const T* Pl, const T* Ql, T dx, T dy, T dz, T* a) {")
    out.append(f"    T Mo[{max(NC1, 1)}];")
    out += ["    " + s for s in mono_lines(P - 1)]
    expr = None
    for j in all_upto(P - 1):
        expr = f"Pl[{idx(j)}] * Mo[{idx(j)}]" if expr is None else f"fma(Pl[{idx(j)}], Mo[{idx(j)}], {expr})"
    out.append(f"    const T pv = {expr};")
    for e in range(3):
        q = None
        for j in all_upto(P - 1):
            q = (f"Ql[{e * NC1 + idx(j)}] * Mo[{idx(j)}]" if q is None
                 else f"fma(Ql[{e * NC1 + idx(j)}], Mo[{idx(j)}], {q})")
        d = ("dx", "dy", "dz")[e]
        out.append(f"    a[{e}] = fma(-{d}, pv, {q});")
    out.append("  }")

    # P2M in the W form: W_k += m (-y)^k / k!   (W_k = (-1)^|k| M_k / k!)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void p2m(T m, T dx, T dy, T dz, T* W) {")
    out.append(f"    T Mo[{NC}];")
    out += ["    " + s for s in mono_lines(P)]
    for k in all_upto(P):
        out.append(f"    W[{idx(k)}] = fma(m, Mo[{idx(k)}], W[{idx(k)}]);")
    out.append("  }")

    # M2M in the W form: W_k(parent) += sum_{i+j=k} W_i(child) (-d)^j / j!,  d = Z_child - Z_parent
    # (called with dx = -d so that Mo holds (-d)^j / j!)
    out.append("  template <typename T>")
    out.append("  __device__ __forceinline__ static void m2m(const T* Ws, T dx, T dy, T dz, T* Wd) {")
    out.append(f"    T Mo[{NC}];")
    out += ["    " + s for s in mono_lines(P)]
    for k in all_upto(P):
        terms = []
        for i in all_upto(sum(k)):
            if i[0] <= k[0] and i[1] <= k[1] and i[2] <= k[2]:
                j = (k[0] - i[0], k[1] - i[1], k[2] - i[2])
                terms.append((idx(i), idx(j)))
        expr = f"Wd[{idx(k)}]"
        for wi, mi in terms:
            expr = f"fma(Ws[{wi}], Mo[{mi}], {expr})"
        out.append(f"    Wd[{idx(k)}] = {expr};")
    out.append("  }")

    out.append("};")
    return out


KNOB_MAX_K = 6  # largest scalar degree K on the GPU (moments to order K + 1 <= 7)


def knob_pairs():
    """(p, K) pairs of the scalar-degree knob built for the GPU: p - 1 < K <= p + 1, K <= KNOB_MAX_K."""
    return [(ps, k) for ps in range(1, PMAX + 1) for k in range(ps, ps + 2) if k <= KNOB_MAX_K]


def gen_knob(PS, K):
    """The projection scalar of the conserving force kept to degree K > PS - 1
    (order-PS standard force realigned, Eq. realign, scalar expanded as in
    Eq. abnab-expansion), as a derivative tensor S_k, |k| <= K, for the
    conserving M2L contraction of order K + 1:
        S(delta) = T_{PS-1}[g](delta) - G_{PS-1}(delta) W_{K-PS+1}(delta),
    with G_{PS-1} the degree-(PS-1) part of g(R + delta) and W_m the Taylor
    polynomial of degree m of w(delta) = (u.delta)/|u|^2 = 1 - (R.u)/|u|^2,
    u = R + delta (no softening in the projection).  So S_k = G_k for
    |k| <= PS - 1, and for PS <= |k| <= K
        S_k = -k! sum_{a + b = k, |a| = PS - 1, |b| >= 1} (G_a / a!) (w_b / b!),
    w_b = -(R.R h_b + sum_d b_d R_d h_{b - e_d}), h_b the derivatives of
    h(u) = 1/|u|^2 at R (radial recurrence with F'_0 = 1/R.R,
    F'_{n+1} = -2 (n+1) F'_n / R.R)."""
    m = K - PS + 1
    out = [f"template <> struct Knob<{PS}, {K}> {{",
           f"  static constexpr int NS = {c_le(K)};",
           "  template <typename T>",
           "  __device__ __forceinline__ static void scalar(T Rx, T Ry, T Rz, const T* G, T* S) {",
           "    const T rr = Rx * Rx + Ry * Ry + Rz * Rz;",
           "    const T irr = T(1) / rr;",
           f"    T H[{m + 1}];",
           "    H[0] = irr;"]
    for n in range(1, m + 1):
        out.append(f"    H[{n}] = {fmt(-2 * n)} * H[{n - 1}] * irr;")
    lines, name = gen_layers(m, 0)
    out += ["    " + l.replace("F[", "H[") for l in lines]
    for k in all_upto(PS - 1):
        out.append(f"    S[{idx(k)}] = G[{idx(k)}];")
    # w_b, 1 <= |b| <= m
    wname = {}
    for b in all_upto(m):
        if sum(b) == 0:
            continue
        terms = [f"rr * {name[(0, b)]}"]
        for d in range(3):
            if b[d] > 0:
                bm = list(b)
                bm[d] -= 1
                c = f"{fmt(b[d])} * " if b[d] > 1 else ""
                terms.append(f"{c}R{AX[d]} * {name[(0, tuple(bm))]}")
        v = f"w_{idx(b)}"
        wname[b] = v
        out.append(f"    const T {v} = -({' + '.join(terms)});")
    import math
    def fact(k):
        return math.factorial(k[0]) * math.factorial(k[1]) * math.factorial(k[2])
    for n in range(PS, K + 1):
        for k in multi(n):
            terms = []
            for a in multi(PS - 1):
                b = (k[0] - a[0], k[1] - a[1], k[2] - a[2])
                if min(b) < 0 or sum(b) < 1:
                    continue
                c = -fact(k) / (fact(a) * fact(b))
                terms.append(f"{fmt(c)} * (G[{idx(a)}] * {wname[b]})")
            out.append(f"    S[{idx(k)}] = {' + '.join(terms)};")
    out.append("  }")
    out.append("};")
    return out


def _count_flops(lines):
    """Floating-point operations in straight-line generated code: an fma
    counts 2, every binary +, - and * written with spaces around it counts 1
    (unary minus and index arithmetic are not counted)."""
    import re
    n = 0
    for ln in lines:
        body = ln.split("=", 1)[1] if "=" in ln else ln
        body = re.sub(r"\[[^\]]*\]", "", body)  # index expressions
        n += 2 * body.count("fma(") + len(re.findall(r" [-+*] ", body))
    return n


def pair_flops(P, variant):
    """Algorithmic FLOPs of one directed far pair in the M2L kernel at order P:
    R, s = |R|^2 + eps^2 and one reciprocal square root (10), the radial
    functions F_1..F_P (2 each), the derivative tensors (generated
    recurrence) and the contraction with the source moments.  variant:
    "standard" (phi derivatives, L_j for |j| >= 1) or "conserving" (g
    derivatives, P and Q'_e)."""
    body = gen_struct(P)
    def fn(name):
        start = next(i for i, l in enumerate(body) if f" {name}(" in l)
        end = next(i for i in range(start + 1, len(body)) if body[i] == "  }")
        return body[start + 1:end]
    prologue = 10 + 2 * P
    if variant == "standard":
        lines = fn("phi_derivs") + fn("m2l_std")
        # the potential term L_0 is not part of the force pass
        lines = [l for l in lines if "if (WITH_POT)" not in l and not l.strip().startswith("L[0] =")]
    else:
        lines = fn("g_derivs") + fn("m2l_cons")
    return prologue + _count_flops(lines)


def main(path=None):
    here = os.path.dirname(os.path.abspath(__file__))
    path = path or os.path.join(here, "expansions_gen.h")
    lines = ["// Generated by gen_expansions.py -- do not edit.",
             "// Cartesian-tensor FMM operators for orders P = 1..%d (see the generator's docstring)." % PMAX,
             "#pragma once",
             "",
             "namespace tfmm {",
             "",
             "template <int P> struct Expansion;",
             ""]
    for P in range(1, PMAX + 1):
        lines += gen_struct(P)
        lines.append("")
    lines.append("// The conserving projection scalar kept to degree K above the default")
    lines.append("// (see gen_knob in the generator).")
    lines.append("template <int PS, int K> struct Knob;")
    for ps, k in knob_pairs():
        lines += gen_knob(ps, k)
        lines.append("")
    lines.append("}  // namespace tfmm")
    text = "\n".join(lines) + "\n"
    with open(path + ".tmp", "w") as f:
        f.write(text)
    os.replace(path + ".tmp", path)
    return path


if __name__ == "__main__":
    print(main(sys.argv[1] if len(sys.argv) > 1 else None))

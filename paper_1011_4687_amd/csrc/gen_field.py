"""Writes field_gen.h: the straight-line code of the field E = -grad V of one
primitive shell pair, one function of each kind per pair angular momentum
L = 0..4.

hermite_field_L{L}(G, X, Y, Z, D, out): with G_n (n = 0..L+1) the scaled
Boys values R^n_000 and X, Y, Z = P - C, runs the McMurchie-Davidson
recursion
    R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v}   (likewise u, v)
to total order L+1 and writes
    out[0] = sum_tuv D_tuv R^0_{tuv}
    out[1] = sum_tuv D_tuv R^0_{t+1,u,v},  out[2] = ... R^0_{t,u+1,v},
    out[3] = ... R^0_{t,u,v+1},
the pair's potential and its gradient with respect to P (= minus the
gradient with respect to the point C).

far_field_L{L}(h, x, y, z, out): in the far field the pair is the finite
multipole (1/R) H(x) with H(x) = sum_abc h_abc x^a y^b z^c, x = X/R^2; this
writes H and its three partial derivatives dH/dx, dH/dy, dH/dz (the caller
forms the gradient of (1/R) H from them).

Components are ordered t ascending, then u, then v (the pair-record order).
Run:  python gen_field.py > field_gen.h
"""
import sys


def comps(L):
    out = []
    for t in range(L + 1):
        for u in range(L + 1 - t):
            for v in range(L + 1 - t - u):
                out.append((t, u, v))
    return out


def name(n, t, u, v):
    return f"r{n}_{t}{u}{v}"


def emit_near(L, w):
    Lr = L + 1
    w(f"template <typename T>\n__device__ __forceinline__ void hermite_field_L{L}("
      f"const T* G, T X, T Y, T Z, const T* __restrict__ D, T* out) {{\n")
    for n in range(Lr, -1, -1):
        w(f"  const T {name(n, 0, 0, 0)} = G[{n}];\n")
        for (t, u, v) in comps(Lr - n):
            if t + u + v == 0:
                continue
            if t > 0:
                ax, a = "X", t
                prev1 = name(n + 1, t - 1, u, v)
                prev2 = name(n + 1, t - 2, u, v) if t > 1 else None
            elif u > 0:
                ax, a = "Y", u
                prev1 = name(n + 1, t, u - 1, v)
                prev2 = name(n + 1, t, u - 2, v) if u > 1 else None
            else:
                ax, a = "Z", v
                prev1 = name(n + 1, t, u, v - 1)
                prev2 = name(n + 1, t, u, v - 2) if v > 1 else None
            if prev2 is None:
                expr = f"{ax} * {prev1}"
            elif a - 1 == 1:
                expr = f"fma({ax}, {prev1}, {prev2})"
            else:
                expr = f"fma({ax}, {prev1}, T({a - 1}) * {prev2})"
            w(f"  const T {name(n, t, u, v)} = {expr};\n")
    cs = comps(L)
    for j, (dt, du, dv) in enumerate([(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        t, u, v = cs[0]
        w(f"  T a{j} = D[0] * {name(0, t + dt, u + du, v + dv)};\n")
        for k, (t, u, v) in enumerate(cs[1:], start=1):
            w(f"  a{j} = fma(D[{k}], {name(0, t + dt, u + du, v + dv)}, a{j});\n")
    w("  out[0] = a0;\n  out[1] = a1;\n  out[2] = a2;\n  out[3] = a3;\n}\n\n")


def mono(a, b, c):
    return f"m{a}{b}{c}"


def emit_far(L, w):
    idx = {c: k for k, c in enumerate(comps(L))}
    w(f"template <typename T>\n__device__ __forceinline__ void far_field_L{L}("
      f"const T* __restrict__ h, T x, T y, T z, T* out) {{\n")
    if L == 0:
        w("  (void)x; (void)y; (void)z;\n  out[0] = h[0];\n  out[1] = T(0);\n"
          "  out[2] = T(0);\n  out[3] = T(0);\n}\n\n")
        return
    # monomials x^a y^b z^c, a+b+c <= L-1 are needed by the derivatives,
    # up to L by H itself
    for (a, b, c) in comps(L):
        if a + b + c == 0:
            continue
        if c > 0:
            prev, f = mono(a, b, c - 1), "z"
        elif b > 0:
            prev, f = mono(a, b - 1, c), "y"
        else:
            prev, f = mono(a - 1, b, c), "x"
        if prev == "m000":
            w(f"  const T {mono(a, b, c)} = {f};\n")
        else:
            w(f"  const T {mono(a, b, c)} = {prev} * {f};\n")
    # H
    w("  T H = h[0];\n")
    for (a, b, c), k in idx.items():
        if a + b + c == 0:
            continue
        w(f"  H = fma(h[{k}], {mono(a, b, c)}, H);\n")
    # derivatives: dH/dx = sum_{a>=1} a sum_{b,c} h_abc x^(a-1) y^b z^c, grouped by a
    for d, axis in enumerate("xyz"):
        groups = {}
        for (a, b, c), k in idx.items():
            e = (a, b, c)[d]
            if e == 0:
                continue
            lower = [a, b, c]
            lower[d] -= 1
            groups.setdefault(e, []).append((k, tuple(lower)))
        names = []
        for e in sorted(groups):
            gname = f"s{axis}{e}"
            terms = groups[e]
            k0, m0 = terms[0]
            first = f"h[{k0}]" if m0 == (0, 0, 0) else f"h[{k0}] * {mono(*m0)}"
            w(f"  T {gname} = {first};\n")
            for k, m in terms[1:]:
                if m == (0, 0, 0):
                    w(f"  {gname} += h[{k}];\n")
                else:
                    w(f"  {gname} = fma(h[{k}], {mono(*m)}, {gname});\n")
            names.append((e, gname))
        e0, g0 = names[0]
        w(f"  T d{axis} = {g0};\n")
        for e, g in names[1:]:
            w(f"  d{axis} = fma(T({e}), {g}, d{axis});\n")
    w("  out[0] = H;\n  out[1] = dx;\n  out[2] = dy;\n  out[3] = dz;\n}\n\n")


def main():
    w = sys.stdout.write
    w("// Generated by gen_field.py -- do not edit.\n")
    w("// Field of one primitive shell pair: the Hermite recursion to one order\n")
    w("// more than the potential, contracted with D_tuv for the potential and\n")
    w("// its gradient, and the far-field polynomial with its derivatives.\n")
    w("#pragma once\n\n")
    for L in range(5):
        emit_near(L, w)
    for L in range(5):
        emit_far(L, w)


if __name__ == "__main__":
    main()

"""Build-time generator of the constant tables and unrolled SH-product code.

Writes ``generated/shv_constants.h`` and ``generated/shv_gaunt.h`` for the HIP
library.  Everything here is derived from closed forms:

  * real SH normalisation K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and a
    scaled associated-Legendre recurrence in z (index i = l*l + l + m, the
    linearisation of Sec. 3.2);
  * triple-product coefficients C_ijk = integral y_i y_j y_k (Eq. 7) from the
    Wigner 3j symbols (Racah's formula, exact rational arithmetic) and the
    unitary map between complex and real harmonics;
  * clamped-cosine Funk-Hecke eigenvalues A_l (Eqs. 10-11) from the
    Ramamoorthi-Hanrahan closed form;
  * log-cap zonal constants 2 pi / (2l + 1) (Eq. 13 projected about z).

Basis convention: real, orthonormal, no Condon-Shortley phase, y_lm ~ cos(m phi)
for m > 0 and sin(|m| phi) for m < 0.

The generated SH-product code is straight-line: registers cannot be indexed by
data on the GPU, so each sparse contraction is unrolled at compile time with
its coefficients as literals.

Run:  python gen_tables.py <out_dir>
"""
from __future__ import annotations

import math

import numpy as np
import os
import sys
from fractions import Fraction

MAX_BANDS = 8
PI = math.pi


# ----------------------------------------------------------------- Wigner 3j

def _f(n):
    return math.factorial(n)


def wigner3j(j1, j2, j3, m1, m2, m3) -> float:
    if m1 + m2 + m3 != 0:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    tri = Fraction(_f(j1 + j2 - j3) * _f(j1 - j2 + j3) * _f(-j1 + j2 + j3), _f(j1 + j2 + j3 + 1))
    pre = tri * _f(j1 + m1) * _f(j1 - m1) * _f(j2 + m2) * _f(j2 - m2) * _f(j3 + m3) * _f(j3 - m3)
    s = Fraction(0)
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    for k in range(kmin, kmax + 1):
        den = (_f(k) * _f(j3 - j2 + k + m1) * _f(j3 - j1 + k - m2) * _f(j1 + j2 - j3 - k)
               * _f(j1 - k - m1) * _f(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    sign = -1 if (j1 - j2 - m3) % 2 else 1
    # value = sign * sqrt(pre) * s, evaluated as sqrt(pre * s^2) with s's sign
    mag = math.sqrt(float(pre * s * s))
    return sign * (1 if s >= 0 else -1) * mag


def complex_gaunt(l1, m1, l2, m2, l3, m3) -> float:
    """integral Y_l1^m1 Y_l2^m2 Y_l3^m3 (no conjugation, Condon-Shortley phase)."""
    if m1 + m2 + m3 != 0 or (l1 + l2 + l3) % 2:
        return 0.0
    w0 = wigner3j(l1, l2, l3, 0, 0, 0)
    if w0 == 0.0:
        return 0.0
    return math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * PI)) * w0 * wigner3j(l1, l2, l3, m1, m2, m3)


def real_to_complex(l, m):
    """Coefficients u with y_lm = sum_m' u[m'] Y_l^m' (complex dict)."""
    if m == 0:
        return {0: 1.0 + 0j}
    a = abs(m)
    s = (-1) ** a
    if m > 0:
        return {a: s / math.sqrt(2) + 0j, -a: 1 / math.sqrt(2) + 0j}
    return {a: -1j * s / math.sqrt(2), -a: 1j / math.sqrt(2)}


def lm(i):
    l = math.isqrt(i)
    return l, i - l * l - l


def real_gaunt(n_bands):
    """Dict (i, j, k) -> C_ijk (nonzero entries only) for i, j, k < n^2."""
    N = n_bands * n_bands
    out = {}
    for i in range(N):
        li, mi = lm(i)
        ui = real_to_complex(li, mi)
        for j in range(i, N):
            lj, mj = lm(j)
            uj = real_to_complex(lj, mj)
            for k in range(j, N):
                lk, mk = lm(k)
                if (li + lj + lk) % 2 or lk > li + lj or lk < abs(li - lj):
                    continue
                uk = real_to_complex(lk, mk)
                acc = 0j
                for a, ca in ui.items():
                    for b, cb in uj.items():
                        c = -a - b
                        if c in uk:
                            acc += ca * cb * uk[c] * complex_gaunt(li, a, lj, b, lk, c)
                assert abs(acc.imag) < 1e-12, (i, j, k, acc)
                if abs(acc.real) > 1e-13:
                    for p in {(i, j, k), (i, k, j), (j, i, k), (j, k, i), (k, i, j), (k, j, i)}:
                        out[p] = acc.real
    return out


# ----------------------------------------------------------------- basis constants

def dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def norm_c(l, m):
    k = math.sqrt((2 * l + 1) / (4 * PI) * _f(l - m) / _f(l + m))
    return k if m == 0 else math.sqrt(2.0) * k


def recurrence_constants():
    """r_lm = Q_l^m(z) / mu_lm with Q_l^m = d^m P_l / dz^m:
         r_mm = 1, r_{m+1,m} = z, r_lm = z r_{l-1,m} + gamma_lm r_{l-2,m};
       y_lm = lam_lm r_lm T_m(x, y) with T_m = Re/Im (x + i y)^|m|;
       d r_lm / dz = rho_lm r_{l,m+1}."""
    mu = {}
    for m in range(MAX_BANDS + 1):
        mu[(m, m)] = Fraction(dfact(2 * m - 1))
        for l in range(m + 1, MAX_BANDS + 1):
            mu[(l, m)] = mu[(l - 1, m)] * Fraction(2 * l - 1, l - m)
    gamma = [[0.0] * MAX_BANDS for _ in range(MAX_BANDS)]
    lam = [[0.0] * MAX_BANDS for _ in range(MAX_BANDS)]
    rho = [[0.0] * MAX_BANDS for _ in range(MAX_BANDS)]
    for l in range(MAX_BANDS):
        for m in range(l + 1):
            if l >= m + 2:
                gamma[l][m] = float(-Fraction(l + m - 1, l - m) * mu[(l - 2, m)] / mu[(l, m)])
            lam[l][m] = norm_c(l, m) * float(mu[(l, m)])
            rho[l][m] = float(mu[(l, m + 1)] / mu[(l, m)]) if m + 1 <= l else 0.0
    return gamma, lam, rho


def clamped_cosine(l):
    if l == 0:
        return PI
    if l == 1:
        return 2 * PI / 3
    if l % 2:
        return 0.0
    return 2 * PI * (-1) ** (l // 2 - 1) / ((l + 2) * (l - 1)) * _f(l) / (2 ** l * _f(l // 2) ** 2)


N_GROUPS = 4


def parity_groups(n, adjoint, ng=N_GROUPS):
    """Output groups of a squaring (one per wave of the four-wave kernels).
    Cost of a group: forward = its FMAs plus the distinct products e_j e_k it
    needs; adjoint = its terms plus twice the distinct symmetric products
    ob_i e_k it needs.  Start from the classes (l odd, m < 0): the selection
    rules of the real Gaunt coefficients make the products a class needs
    largely shared within it.  Then take best-improvement single moves while
    they lower the largest group cost.  Deterministic."""
    import collections
    N = n * n
    C = real_gaunt(n)
    ft = {i: [] for i in range(N)}
    at = {m: set() for m in range(N)}
    for (i, j, k) in C:
        if j <= k:
            ft[i].append((j, k))
        at[j].add((i, k) if i <= k else (k, i))
    at = {m: sorted(v) for m, v in at.items()}
    grp = []
    for i in range(N):
        l, m = lm(i)
        grp.append((2 * (l % 2) + (1 if m < 0 else 0)) % ng)
    fc = [collections.Counter() for _ in range(ng)]
    ac = [collections.Counter() for _ in range(ng)]
    fterm, aterm = [0] * ng, [0] * ng

    def add(i, g, sgn):
        if sgn > 0:
            fc[g].update(ft[i])
            ac[g].update(at[i])
        else:
            fc[g].subtract(ft[i])
            ac[g].subtract(at[i])
            fc[g] += collections.Counter()
            ac[g] += collections.Counter()
        fterm[g] += sgn * len(ft[i])
        aterm[g] += sgn * len(at[i])

    for i in range(N):
        add(i, grp[i], 1)

    def score():
        if adjoint:
            return max(aterm[g] + 2 * len(ac[g]) for g in range(ng))
        return max(fterm[g] + len(fc[g]) for g in range(ng))

    cur = score()
    while True:
        best = None
        for i in range(N):
            a = grp[i]
            for b in range(ng):
                if b == a:
                    continue
                add(i, a, -1)
                add(i, b, 1)
                s = score()
                add(i, b, -1)
                add(i, a, 1)
                if s < cur and (best is None or s < best[0]):
                    best = (s, i, b)
        if best is None:
            break
        cur, i, b = best
        add(i, grp[i], -1)
        add(i, b, 1)
        grp[i] = b
    return [sorted(i for i in range(N) if grp[i] == g) for g in range(ng)]


def forward_groups(n, ng=N_GROUPS):
    return parity_groups(n, False, ng)


def adjoint_groups(n, ng=N_GROUPS):
    """Also the canonical grouping of the backward's sums."""
    return parity_groups(n, True, ng)


# ----------------------------------------------------------------- emission

def flit(x: float) -> str:
    """float literal that round-trips the nearest float32."""
    import struct
    f = struct.unpack("f", struct.pack("f", x))[0]
    s = repr(f)
    if "e" not in s and "." not in s:
        s += ".0"
    return s + "f"


def emit_constants(path):
    gamma, lam, rho = recurrence_constants()
    lines = ["// Generated by gen_tables.py: SH recurrence and transfer constants.",
             "#pragma once", "", f"#define SHV_MAX_BANDS {MAX_BANDS}", ""]

    def table2(name, t):
        lines.append(f"static constexpr float {name}[{MAX_BANDS}][{MAX_BANDS}] = {{")
        for row in t:
            lines.append("  {" + ", ".join(flit(v) for v in row) + "},")
        lines.append("};")

    table2("SHV_GAMMA", gamma)
    table2("SHV_LAMBDA", lam)
    table2("SHV_RHO", rho)
    lines.append(f"static constexpr float SHV_AHAT[{MAX_BANDS}] = {{"
                 + ", ".join(flit(clamped_cosine(l)) for l in range(MAX_BANDS)) + "};")
    # log-cap zonal: g_l(t) = -eps * 2 pi/(2l+1) * (P_{l-1}(t) - P_{l+1}(t))
    lines.append(f"static constexpr float SHV_CAPK[{MAX_BANDS}] = {{"
                 + ", ".join(flit(-2 * PI / (2 * l + 1)) for l in range(MAX_BANDS)) + "};")
    # Bonnet: P_{l+1} = (2l+1)/(l+1) t P_l - l/(l+1) P_{l-1}
    lines.append(f"static constexpr float SHV_BONNET_A[{MAX_BANDS + 1}] = {{"
                 + ", ".join(flit((2 * l + 1) / (l + 1)) for l in range(MAX_BANDS + 1)) + "};")
    lines.append(f"static constexpr float SHV_BONNET_B[{MAX_BANDS + 1}] = {{"
                 + ", ".join(flit(l / (l + 1)) for l in range(MAX_BANDS + 1)) + "};")
    lines.append("static constexpr float SHV_SQRT_4PI = " + flit(math.sqrt(4 * PI)) + ";")
    lines.append("static constexpr float SHV_INV_SQRT_4PI = " + flit(1 / math.sqrt(4 * PI)) + ";")
    lines.append("static constexpr float SHV_INV_8PI = " + flit(1 / (8 * PI)) + ";")
    lines.append("static constexpr float SHV_INV_4PI = " + flit(1 / (4 * PI)) + ";")
    lines.append("static constexpr float SHV_TWO_PI = " + flit(2 * PI) + ";")
    open(path, "w").write("\n".join(lines) + "\n")


def transfer_support(n):
    """Coefficient indices where the clamped-cosine transfer can be nonzero."""
    return [i for i in range(n * n) if clamped_cosine(lm(i)[0]) != 0.0]


def emit_gaunt(path):
    L = ["// Generated by gen_tables.py: unrolled sparse SH triple products.",
         "// C_ijk = integral y_i y_j y_k from Wigner 3j symbols; straight-line code",
         "// because GPU registers cannot be indexed by data.",
         "#pragma once", ""]
    tables = []
    for n in range(1, MAX_BANDS + 1):
        N = n * n
        C = real_gaunt(n)
        nnz = len(C)
        sym = sorted((i, j, k) for (i, j, k) in C if j <= k)
        L.append(f"// n = {n}: {nnz} nonzero C_ijk, {len(sym)} with j <= k")
        L.append(f"#define SHV_GAUNT_NNZ_{n} {nnz}")

        # o = e * e (symmetric squaring)
        L.append(f"__device__ __forceinline__ void shv_square_{n}(const float* __restrict__ e, float* __restrict__ o) {{")
        touched = set()
        pairs = {}
        for (i, j, k) in sym:
            pairs.setdefault((j, k), []).append(i)
        for (j, k) in sorted(pairs):
            L.append(f"  {{ const float t = e[{j}] * e[{k}];")
            for i in pairs[(j, k)]:
                c = C[(i, j, k)] * (2.0 if j < k else 1.0)
                if i in touched:
                    L.append(f"    o[{i}] = fmaf({flit(c)}, t, o[{i}]);")
                else:
                    L.append(f"    o[{i}] = {flit(c)} * t;")
                    touched.add(i)
            L.append("  }")
        for i in range(N):
            if i not in touched:
                L.append(f"  o[{i}] = 0.0f;")
        L.append("}")

        # eb = 2 * (ob * e): adjoint of o = e * e
        L.append(f"__device__ __forceinline__ void shv_square_adj_{n}(const float* __restrict__ ob, const float* __restrict__ e, float* __restrict__ eb) {{")
        touched = set()
        upairs = {}
        for (j, i, k) in C:           # eb_j += 2 C_jik ob_i e_k
            if i <= k:
                upairs.setdefault((i, k), []).append(j)
        for (i, k) in sorted(upairs):
            if i == k:
                L.append(f"  {{ const float u = ob[{i}] * e[{i}];")
            else:
                L.append(f"  {{ const float u = fmaf(ob[{i}], e[{k}], ob[{k}] * e[{i}]);")
            for j in sorted(upairs[(i, k)]):
                c = 2.0 * C[(j, i, k)]
                if j in touched:
                    L.append(f"    eb[{j}] = fmaf({flit(c)}, u, eb[{j}]);")
                else:
                    L.append(f"    eb[{j}] = {flit(c)} * u;")
                    touched.add(j)
            L.append("  }")
        for j in range(N):
            if j not in touched:
                L.append(f"  eb[{j}] = 0.0f;")
        L.append("}")

        # Per-group variants for kernels that split one receiver's squaring
        # over several waves: group g computes only its outputs, with exactly
        # the per-output term order of the full functions above.
        groups = forward_groups(n)
        agroups = adjoint_groups(n)
        for name, grs in (("SHV_FGRP", groups), ("SHV_GRP", agroups)):
            gid = [0] * N
            for g, members in enumerate(grs):
                for i in members:
                    gid[i] = g
            L.append(f"static constexpr unsigned char {name}_{n}[{N}] = {{" + ",".join(map(str, gid)) + "};")
        for g, members in enumerate(groups):
            mem = set(members)
            L.append(f"__device__ __forceinline__ void shv_square_{n}_g{g}(const float* __restrict__ e, float* __restrict__ o) {{")
            touched = set()
            for (j, k) in sorted(pairs):
                outs = [i for i in pairs[(j, k)] if i in mem]
                if not outs:
                    continue
                L.append(f"  {{ const float t = e[{j}] * e[{k}];")
                for i in outs:
                    c = C[(i, j, k)] * (2.0 if j < k else 1.0)
                    if i in touched:
                        L.append(f"    o[{i}] = fmaf({flit(c)}, t, o[{i}]);")
                    else:
                        L.append(f"    o[{i}] = {flit(c)} * t;")
                        touched.add(i)
                L.append("  }")
            for i in members:
                if i not in touched:
                    L.append(f"  o[{i}] = 0.0f;")
            L.append("}")
        for g, members in enumerate(agroups):
            mem = set(members)
            L.append(f"__device__ __forceinline__ void shv_square_adj_{n}_g{g}(const float* __restrict__ ob, const float* __restrict__ e, float* __restrict__ eb) {{")
            touched = set()
            for (i, k) in sorted(upairs):
                outs = [j for j in sorted(upairs[(i, k)]) if j in mem]
                if not outs:
                    continue
                if i == k:
                    L.append(f"  {{ const float u = ob[{i}] * e[{i}];")
                else:
                    L.append(f"  {{ const float u = fmaf(ob[{i}], e[{k}], ob[{k}] * e[{i}]);")
                for j in outs:
                    c = 2.0 * C[(j, i, k)]
                    if j in touched:
                        L.append(f"    eb[{j}] = fmaf({flit(c)}, u, eb[{j}]);")
                    else:
                        L.append(f"    eb[{j}] = {flit(c)} * u;")
                        touched.add(j)
                L.append("  }")
            for j in members:
                if j not in touched:
                    L.append(f"  eb[{j}] = 0.0f;")
            L.append("}")

        # sparse table grouped by (j, k) for building M(L)_jk = sum_i L_i C_ijk
        rows = [[] for _ in range(N * N)]
        for (i, j, k), c in C.items():
            rows[j * N + k].append((i, c))
        ptr = [0]
        ent_i, ent_c = [], []
        for r in rows:
            for i, c in sorted(r):
                ent_i.append(i)
                ent_c.append(c)
            ptr.append(len(ent_i))
        tables.append((n, ptr, ent_i, ent_c))
        L.append("")

    L.append("// (j, k)-grouped sparse C for building M(L); CSR over j*N + k.")
    for n, ptr, ei, ec in tables:
        L.append(f"__device__ const int shv_mtab_ptr_{n}[{len(ptr)}] = {{" + ",".join(map(str, ptr)) + "};")
        L.append(f"__device__ const unsigned char shv_mtab_idx_{n}[{max(len(ei), 1)}] = {{" + ",".join(map(str, ei or [0])) + "};")
        L.append(f"__device__ const float shv_mtab_val_{n}[{max(len(ec), 1)}] = {{" + ",".join(flit(c) for c in (ec or [0.0])) + "};")
    L.append("")
    L.append("// Lighting-gradient contraction Lbar_i = sum_{j, kk} C_{i j k(kk)} Q[j][kk],")
    L.append("// Q over the transfer support (kk indexes the support); entries j * 32 + kk, row i's")
    L.append("// entries split over 4 threads (entry e of the row to thread e mod 4), padded per thread.")
    for n in range(1, MAX_BANDS + 1):
        N = n * n
        C = real_gaunt(n)
        supp = transfer_support(n)
        pos = {k: kk for kk, k in enumerate(supp)}
        rows = [[] for _ in range(N)]
        for (i, j, k), c in C.items():
            if k in pos:
                rows[i].append((j * 32 + pos[k], c))
        ptr, ent, val = [0], [], []
        for r in rows:
            for e, c in sorted(r):
                ent.append(e)
                val.append(c)
            ptr.append(len(ent))
        # Padded per-thread layout: thread (i, part) of the contraction takes
        # the entries ptr[i] + part, + 4, ... in order, as slots 0, 1, ...;
        # every (i, part) gets the same slot count (unused slots: entry 0,
        # value 0, beyond the count) so its loads can all be issued at once.
        slots = max([(ptr[i + 1] - ptr[i] - part + 3) // 4 for i in range(N) for part in range(4)] + [1])
        pent, pval, pcnt = [], [], []
        for i in range(N):
            for part in range(4):
                es = list(range(ptr[i] + part, ptr[i + 1], 4))
                pcnt.append(len(es))
                pent += [ent[e] for e in es] + [0] * (slots - len(es))
                pval += [val[e] for e in es] + [0.0] * (slots - len(es))
        L.append(f"static constexpr int SHV_LTAB_SLOTS_{n} = {slots};")
        L.append(f"__device__ const int shv_ltab_cnt_{n}[{len(pcnt)}] = {{" + ",".join(map(str, pcnt)) + "};")
        L.append(f"__device__ const unsigned short shv_ltab_pent_{n}[{len(pent)}] = {{" + ",".join(map(str, pent)) + "};")
        L.append(f"__device__ const float shv_ltab_pval_{n}[{len(pval)}] = {{" + ",".join(flit(c) for c in pval) + "};")
    L.append("")
    L.append("// Quadrature of the projected exponential: Gauss-Legendre nodes and weights in z,")
    L.append("// 4n of them for n bands (the rule of degree 8n - 1 with 8n uniform azimuths).")
    for n in range(1, MAX_BANDS + 1):
        z, wz = np.polynomial.legendre.leggauss(4 * n)
        L.append(f"__device__ const float shv_quad_z_{n}[{4 * n}] = {{" + ",".join(flit(v) for v in z) + "};")
        L.append(f"__device__ const float shv_quad_w_{n}[{4 * n}] = {{" + ",".join(flit(v) for v in wz) + "};")
    L.append("")
    for n in range(1, MAX_BANDS + 1):
        supp = transfer_support(n)
        L.append(f"static constexpr int SHV_HSUPP_COUNT_{n} = {len(supp)};")
        L.append(f"static constexpr int SHV_HSUPP_{n}[{len(supp)}] = {{" + ",".join(map(str, supp)) + "};")
    open(path, "w").write("\n".join(L) + "\n")


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "generated")
    os.makedirs(out, exist_ok=True)
    # self-checks of the derivation (selection rules and DC row)
    for n, nnz in ((4, 353), (6, 2907), (8, 12868)):
        C = real_gaunt(n)
        assert len(C) == nnz, (n, len(C))
        for j in range(n * n):
            assert abs(C.get((0, j, j), 0.0) - 1 / math.sqrt(4 * PI)) < 1e-14
    emit_constants(os.path.join(out, "shv_constants.h"))
    emit_gaunt(os.path.join(out, "shv_gaunt.h"))


if __name__ == "__main__":
    main()

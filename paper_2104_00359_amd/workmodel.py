"""Algorithmic work per unit for each kernel (used for roofline figures).

Counting rule: one floating-point add, multiply, square root, reciprocal
square root or exponential = 1 flop; a fused multiply-add = 2 flops.  The
counts are those of the minimal operation graph of the formulation the
kernels implement (polynomial SH basis, sparse triple products); lane-level
overheads (index arithmetic, cross-lane reductions, tail lanes) are not
counted.  Units: one (receiver, sphere) pair for the pair kernels, one
receiver for the per-receiver kernels.
"""
from __future__ import annotations

import functools
import os
import sys


def _tri(n):
    return n * (n - 1) // 2


def pair_fwd_flops(n: int) -> int:
    geom = 20                                   # c - x, |v|^2, rsqrt, s, r/d, 1 - s^2, sqrt, u = s^2/(1+t)
    leg = 5 * max(n - 1, 0)                     # residual Bonnet steps R_2 .. R_n
    cap = 2 * n - 1                             # g_0 = K_0 u, g_l = K_l (R_{l+1} - R_{l-1})
    cs = 6 * max(n - 2, 0)                      # Re/Im (x + i y)^m, m = 2 .. n-1
    rec = 3 * max(n - 2, 0) * max(n - 1, 0) // 2  # r_l^m three-term steps
    u = _tri(n)                                 # g_l r_l^m for l > m
    acc = n + 3 + 4 * _tri(n)                   # m = 0 adds (compensated DC), m > 0 two FMAs each
    return geom + leg + cap + cs + rec + u + acc


def pair_bwd_flops(n: int) -> int:
    base = 20 + 5 * max(n - 1, 0) + 2 * n - 1 + 6 * max(n - 2, 0) + 3 * max(n - 2, 0) * max(n - 1, 0) // 2
    vw = 3 * _tri(n) + n                        # g_l r and (1 - R_l) r
    m0 = 2 * n                                  # t-derivative sum of the m = 0 column
    lm = 10 * _tri(n) + 2 * _tri(max(n - 1, 0))  # X, T (4 FMAs) and Z sums per (l, m >= 1)
    comb = 4 + 18 * max(n - 1, 0)               # per-order combination into Gx, Gy, Gz, Gt
    chain = 26 + 3 + 4                          # tangent projection, t chain, receiver / sphere sums
    return base + vw + m0 + lm + comb + chain


@functools.lru_cache(maxsize=None)
def _gaunt_counts(n: int):
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    if here not in sys.path:
        sys.path.insert(0, here)
    import gen_tables  # the library's own table generator
    C = gen_tables.real_gaunt(n)
    sym = [(i, j, k) for (i, j, k) in C if j <= k]
    pairs = {(j, k) for (_, j, k) in sym}
    upairs = {(i, k) for (_, i, k) in C if i <= k}
    supp = set(gen_tables.transfer_support(n))
    vh = [(i, j, k) for (i, j, k) in C if k in supp]
    vh_pairs = {(j, k) for (_, j, k) in vh}
    return dict(nnz=len(C), sym=len(sym), pairs=len(pairs), upairs=len(upairs),
                diag=sum(1 for (i, k) in upairs if i == k), vh=len(vh), vh_pairs=len(vh_pairs),
                supp=len(supp))


def square_flops(n: int) -> int:
    c = _gaunt_counts(n)
    return c["pairs"] + 2 * c["sym"]


def square_adj_flops(n: int) -> int:
    c = _gaunt_counts(n)
    off = c["upairs"] - c["diag"]
    return c["diag"] + 3 * off + 2 * c["sym"]


def exp_fwd_flops(n: int, k: int) -> int:
    N = n * n
    prologue = 3 * N + 2 * N + 4                # scale, |G|^2, exp, a * G
    return prologue + k * square_flops(n) + N + 1


def exp_bwd_flops(n: int, k: int) -> int:
    N = n * n
    return 3 * N + 2 + k * square_adj_flops(n) + 2 * N + 5 * N


def shade_fwd_flops(n: int) -> int:
    c = _gaunt_counts(n)
    N = n * n
    return 12 + 3 * N + c["supp"] * (2 * N + 2) + 1


def shade_bwd_flops(n: int) -> int:
    c = _gaunt_counts(n)
    N = n * n
    h = 12 + 3 * N
    mv = c["supp"] * (2 * N + 3)
    vbar = N * (2 * c["supp"] + 1)
    nbar = 10 * N + 15
    lbar = c["supp"] + 2 * N * c["supp"]        # w H, then the Q GEMM (contraction with C is per call)
    return h + mv + vbar + nbar + lbar


def shade_ch_fwd_flops(n: int, channels: int) -> int:
    """Several channels: the transfer once, V^T M_c H per channel."""
    c = _gaunt_counts(n)
    N = n * n
    return 12 + 3 * N + channels * (c["supp"] * (2 * N + 2) + 1)


def shade_ch_bwd_flops(n: int, channels: int) -> int:
    """Several channels: the transfer and the normal cotangent once, the
    shading value, V and H cotangents and the lighting GEMM per channel (the
    channel sums of the V and H cotangents are one add per entry)."""
    c = _gaunt_counts(n)
    N = n * n
    h = 12 + 3 * N
    mv = c["supp"] * (2 * N + 4)
    vbar = N * (2 * c["supp"] + 2)
    nbar = 10 * N + 15
    lbar = c["supp"] + 2 * N * c["supp"]
    return h + nbar + channels * (mv + vbar + lbar)


def quad_nodes(n: int) -> int:
    """Nodes of the quadrature exponential's rule (4n x 8n)."""
    return 32 * n * n


def exp_quad_fwd_flops(n: int) -> int:
    """Per receiver: f = Fhat Y over the nodes and V = (w exp f) Y^T, two
    N x Q products, plus one exponential and one weight multiply per node."""
    N, Q = n * n, quad_nodes(n)
    return 2 * (2 * N * Q) + 2 * Q


def exp_quad_bwd_flops(n: int) -> int:
    """Per receiver: f and g = Vbar Y, then Fbar = (w exp f g) Y^T: three
    N x Q products, plus the exponential and two multiplies per node."""
    N, Q = n * n, quad_nodes(n)
    return 3 * (2 * N * Q) + 3 * Q


def exp_taylor_fwd_flops(n: int, k: int, K: int) -> int:
    """Per receiver: the DC split and scaling (2 N), K Horner steps (one
    sparse product each, returned doubled, and its scale), k squarings and
    the final exp(c) scale."""
    N = n * n
    return 2 * N + K * (square_adj_flops(n) + N) + k * square_flops(n) + N + 1


def exp_taylor_bwd_flops(n: int, k: int, K: int) -> int:
    """Per receiver: cbar and exp(c) Vbar (3 N), k adjoint squarings, the
    Horner adjoint (two sparse products per step but one in the last, each
    with its scale / accumulation) and the weights W (2 N)."""
    N = n * n
    return 3 * N + k * square_adj_flops(n) + (2 * K - 1) * (square_adj_flops(n) + 2 * N) + 2 * N


def prod_fwd_flops(n: int) -> int:
    """Per (receiver, sphere) step of the direct product chain: the pair's
    blocker vector (the pair forward's basis work plus one LAMBDA multiply per
    coefficient), one sparse product V * h (the generated product, which
    returns 2 V * h) and the update V + beta/2 (2 V * h)."""
    N = n * n
    return pair_fwd_flops(n) + N + square_adj_flops(n) + 2 * N


def prod_bwd_flops(n: int) -> int:
    """Per step of the chain's adjoint: the blocker vector again, the two
    sparse products Vbar * V_in and Vbar * h with their scale and update, the
    pair weights W and RHO W, and the pair adjoint."""
    N = n * n
    return (pair_fwd_flops(n) + N) + 2 * square_adj_flops(n) + 3 * N + 2 * N + pair_bwd_flops(n)


def envmap_pixel_flops(n: int) -> int:
    """One map pixel: sin and cos of its azimuth, the direction (3), the
    polynomial SH basis (powers of x + i y, three-term recurrences in z, one
    normalising multiply per coefficient) and one FMA per coefficient."""
    N = n * n
    basis = 6 * max(n - 1, 0) + 3 * n * (n - 1) // 2 + N
    return 2 + 3 + basis + 2 * N


# Bytes each kernel must move to / from HBM per unit (FP32).
def exp_fwd_bytes(n: int, k: int, nchunks: int) -> int:
    N = n * n
    return 4 * (nchunks * N + N + 1 + k * N)


def pair_fwd_bytes_per_receiver(n: int, nchunks: int) -> int:
    return 4 * (3 * nchunks + n * n * nchunks)


def exp_shade_bwd_bytes(n: int, k: int) -> int:
    """Algorithmic HBM bytes per receiver of the fused exponential + shading
    adjoint: it reads the radiance cotangent, V, the saved c and E_0 ..
    E_{k-1}, the normal and the albedo, and writes W (the cotangent of F'),
    the normal and albedo gradients and its share of the per-tile lighting
    partials (N floats per 64 receivers)."""
    N = n * n
    reads = 4 * (1 + N + (1 + k * N) + 3 + 1)
    writes = 4 * (N + 3 + 1) + 4 * N / 64
    return int(round(reads + writes))


def kernel_work(name: str, n: int, k: int, P: int, S: int, channels: int = 1, pixels: int = 0, order: int = 0):
    """(flops, unit count) of one launch of kernel ``name`` (``channels``
    for the multi-channel shading kernels, ``pixels`` = C H W for the
    environment-map projection, ``order`` = K of the Taylor exponential)."""
    if name == "exp_taylor_fwd":
        return exp_taylor_fwd_flops(n, k, order) * P, P
    if name == "exp_taylor_bwd":
        return exp_taylor_bwd_flops(n, k, order) * P, P
    if name == "shade_ch_fwd":
        return shade_ch_fwd_flops(n, channels) * P, P
    if name == "shade_ch_bwd":
        return shade_ch_bwd_flops(n, channels) * P, P
    if name == "envmap_rows":
        return envmap_pixel_flops(n) * pixels, pixels
    if name == "exp_quad_fwd":
        return exp_quad_fwd_flops(n) * P, P
    if name == "exp_quad_bwd":
        return exp_quad_bwd_flops(n) * P, P
    if name in ("prod_fwd", "prod_fwd_states"):
        return prod_fwd_flops(n) * P * S, P * S
    if name == "prod_bwd":
        return prod_bwd_flops(n) * P * S, P * S
    if name == "pair_fwd":
        return pair_fwd_flops(n) * P * S, P * S
    if name == "pair_bwd":
        return pair_bwd_flops(n) * P * S, P * S
    if name == "exp_fwd":
        return exp_fwd_flops(n, k) * P, P
    if name == "exp_bwd":
        return exp_bwd_flops(n, k) * P, P
    if name == "shade_fwd":
        return shade_fwd_flops(n) * P, P
    if name == "shade_bwd":
        return shade_bwd_flops(n) * P, P
    if name == "exp_shade_fwd":
        return (exp_fwd_flops(n, k) + shade_fwd_flops(n)) * P, P
    if name == "exp_shade_bwd":
        return (exp_bwd_flops(n, k) + shade_bwd_flops(n)) * P, P
    return None, None


BATCH_KERNELS = {"batch_pair_fwd": "pair_fwd", "batch_pair_bwd": "pair_bwd", "batch_exp_shade_fwd": "exp_shade_fwd",
                 "batch_exp_shade_bwd": "exp_shade_bwd"}


def batch_work(name: str, scenes):
    """(flops, unit count) of all launches of batched kernel ``name`` in one
    batched call over ``scenes`` (tuples (n, k, P, S)).  A name carrying a
    band count ("batch_pair_bwd/n8", "batch_exp_shade_fwd/n4/one") counts the
    scenes with that many bands only."""
    parts = name.split("/")
    single = BATCH_KERNELS.get(parts[0])
    if single is None:
        return None, None
    only = int(parts[1][1:]) if len(parts) > 1 and parts[1].startswith("n") else None
    flops = units = 0
    for n, k, P, S in scenes:
        if only is not None and n != only:
            continue
        f, u = kernel_work(single, n, k, P, S)
        flops += f
        units += u
    return flops, units

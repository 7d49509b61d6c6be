"""Seeded synthetic inputs for the closed-shell (T) energy.

This module only draws and assembles inputs; it contains none of the (T)
arithmetic.  It serves both the HIP path and the CPU oracle, which share
nothing else.

Workload shape (stand-in for the paper's alanine-chain inputs, Sec. 4; the
paper itself fills its arrays with arbitrary numbers when timing):

* n = o + v spatial orbitals, orbitals 0..o-1 occupied, o..n-1 virtual.
* Density-fitting factor B[Q, p, q] ~ N(0, 0.1^2), naux = 3 n, made symmetric
  in (p, q) so that the integrals carry the real-orbital 8-fold symmetry the
  closed-shell formulas assume (Sec. 2.1, eq. eri_sym_decomp gives the form
  (pq|rs) = sum_Q B^Q_pq B^Q_rs).
* eps_occ ~ U[-2.0, -0.3], eps_virt ~ U[0.2, 5.0]; t1 ~ N(0, 1e-3^2).
* t2 = first-order (MP2) doubles, t^ab_ij = (ia|jb) / (e_i + e_j - e_a - e_b).

Array layouts (C row-major, float64), Mulliken notation:
  eps_o[o], eps_v[v], t1[i][a], t2[i][j][a][b] = t^ab_ij,
  vvvo[a][b][c][i] = (ab|ci), ovoo[i][a][j][k] = (ia|jk), ovov[i][a][j][b] = (ia|jb).

Two generators:
* ``make_problem`` (numpy PCG64, float64 throughout) for every size the host
  can hold; draw order B, eps_o, eps_v, t1 from ``default_rng(seed)``.
* ``make_problem_device`` for the large workloads whose (vv|vo) block does
  not fit host memory: the same draws on the host, the same float64 products
  formed on the GPU with torch (summation order may differ in the last bit).
"""
from __future__ import annotations

import numpy as np

# sizes of the five workloads: (o, v)
CONFIGS = {
    "C0": dict(o=6, v=30),
    "C1": dict(o=20, v=200),
    "C2": dict(o=30, v=400),
    "C3": dict(o=40, v=600),
}
# RI-MP2 workloads: the smallest alanine-chain size of the paper's RI-MP2
# timings (o, v, naux), and a small one for parity tests.
MP2_CONFIGS = {
    "M0": dict(o=8, v=60, naux=150),
    "M1": dict(o=119, v=2546, naux=5852),
}
# Physically scaled variant: B multiplied by a factor so that |E(T)| of the
# workload is of physical size (about 0.1-0.3 Eh for seed 0) instead of the
# 1e2-1e13 Eh the unscaled recipe gives.  Integrals scale as s^2, the MP2
# doubles as s^2, W as s^4, so E[4] scales as s^8 and E[5] as s^6.
PHYSICAL_B_SCALE = {"C0": 0.4, "C1": 0.06, "C2": 0.03, "C3": 0.02}
BATCH_NPROB = 64
BATCH_O_RANGE = (4, 16)
BATCH_V_RANGE = (40, 160)


def _symmetrize_B(B: np.ndarray) -> np.ndarray:
    """Copy the upper triangle (p <= q) of each B^Q onto the lower one."""
    up = np.triu(B)
    return up + np.triu(B, 1).transpose(0, 2, 1)


def draw_factors(o: int, v: int, seed: int, naux: int | None = None, b_scale: float = 1.0):
    """Draw (B, eps_o, eps_v, t1) in the fixed order of the recipe; B is
    multiplied by ``b_scale`` after the draw (same random stream)."""
    n = o + v
    naux = 3 * n if naux is None else naux
    rng = np.random.default_rng(seed)
    B = _symmetrize_B(rng.normal(0.0, 0.1, size=(naux, n, n)))
    if b_scale != 1.0:
        B *= b_scale
    eps_o = rng.uniform(-2.0, -0.3, size=o)
    eps_v = rng.uniform(0.2, 5.0, size=v)
    t1 = rng.normal(0.0, 1e-3, size=(o, v))
    return B, eps_o, eps_v, t1


def full_eri(B: np.ndarray) -> np.ndarray:
    """(pq|rs) over all n orbitals, symmetrized to exact 8-fold symmetry.

    Only for tiny n (n^4 doubles)."""
    g = np.einsum("Qpq,Qrs->pqrs", B, B, optimize=True)
    g = 0.5 * (g + g.transpose(1, 0, 2, 3))
    g = 0.5 * (g + g.transpose(0, 1, 3, 2))
    g = 0.5 * (g + g.transpose(2, 3, 0, 1))
    return g


def _mp2_doubles(ovov: np.ndarray, eps_o: np.ndarray, eps_v: np.ndarray) -> np.ndarray:
    """t2[i,j,a,b] = (ia|jb) / (e_i + e_j - e_a - e_b)."""
    den = (eps_o[:, None, None, None] + eps_o[None, :, None, None]
           - eps_v[None, None, :, None] - eps_v[None, None, None, :])
    return np.ascontiguousarray(ovov.transpose(0, 2, 1, 3) / den)


def make_problem(o: int, v: int, seed: int = 0, naux: int | None = None,
                 with_eri: bool = False, with_df: bool = False, b_scale: float = 1.0) -> dict:
    """Host float64 problem.  ``with_eri`` also returns the full 8-fold
    symmetric ERI tensor ``eri`` (tiny sizes), from which every block is
    sliced so the blocks agree with it bit for bit.  ``with_df`` also returns
    the density-fitting factors with the auxiliary index fastest,
    bvv[a][b][Q] = B^Q_ab and bvo[c][i][Q] = B^Q_ci, and ``naux``.
    ``b_scale`` multiplies B (see PHYSICAL_B_SCALE)."""
    B, eps_o, eps_v, t1 = draw_factors(o, v, seed, naux, b_scale)
    O = slice(0, o)
    V = slice(o, o + v)
    out = dict(nocc=o, nvirt=v, eps_o=eps_o, eps_v=eps_v, t1=np.ascontiguousarray(t1))
    if with_df:
        out["naux"] = B.shape[0]
        out["bvv"] = np.ascontiguousarray(B[:, V, V].transpose(1, 2, 0))
        out["bvo"] = np.ascontiguousarray(B[:, V, O].transpose(1, 2, 0))
    if with_eri:
        g = full_eri(B)
        ovov = np.ascontiguousarray(g[O, V, O, V])
        ovoo = np.ascontiguousarray(g[O, V, O, O])
        vvvo = np.ascontiguousarray(g[V, V, V, O])
        out["eri"] = g
    else:
        Bov = B[:, O, V]
        Bvv = B[:, V, V]
        Boo = B[:, O, O]
        ovov = np.tensordot(Bov, Bov, axes=([0], [0]))            # [i,a,j,b]
        ovov = 0.5 * (ovov + ovov.transpose(2, 3, 0, 1))          # (ia|jb) = (jb|ia)
        ovoo = np.tensordot(Bov, Boo, axes=([0], [0]))            # [i,a,j,k]
        ovoo = 0.5 * (ovoo + ovoo.transpose(0, 1, 3, 2))          # (ia|jk) = (ia|kj)
        Bvo = B[:, V, O]
        vvvo = np.tensordot(Bvv, Bvo, axes=([0], [0]))            # [a,b,c,i]
        vvvo = 0.5 * (vvvo + vvvo.transpose(1, 0, 2, 3))          # (ab|ci) = (ba|ci)
        ovov = np.ascontiguousarray(ovov)
        ovoo = np.ascontiguousarray(ovoo)
        vvvo = np.ascontiguousarray(vvvo)
    out["ovov"] = ovov
    out["ovoo"] = ovoo
    out["vvvo"] = vvvo
    out["t2"] = _mp2_doubles(ovov, eps_o, eps_v)
    return out


def batch_shapes(seed: int = 0, nprob: int = BATCH_NPROB):
    """(o_p, v_p) for the batched workload: o ~ U{4..16}, v ~ U{40..160}."""
    rng = np.random.default_rng(seed)
    os_ = rng.integers(BATCH_O_RANGE[0], BATCH_O_RANGE[1] + 1, size=nprob)
    vs_ = rng.integers(BATCH_V_RANGE[0], BATCH_V_RANGE[1] + 1, size=nprob)
    return [(int(a), int(b)) for a, b in zip(os_, vs_)]


def make_batch(seed: int = 0, nprob: int = BATCH_NPROB) -> list[dict]:
    """Batched workload: problem p has the drawn shape and uses seed + p."""
    return [make_problem(o, v, seed + p) for p, (o, v) in enumerate(batch_shapes(seed, nprob))]


FIELDS = ("eps_o", "eps_v", "t1", "t2", "vvvo", "ovoo", "ovov")
DF_FIELDS = ("bvv", "bvo")


def to_device(prob: dict, device="cuda"):
    """Copy the float64 arrays of a host problem into torch tensors."""
    import torch
    out = dict(nocc=prob["nocc"], nvirt=prob["nvirt"])
    if "naux" in prob:
        out["naux"] = prob["naux"]
    for f in FIELDS + DF_FIELDS:
        if f in prob:
            out[f] = torch.from_numpy(np.ascontiguousarray(prob[f])).to(device)
    return out


def make_problem_device(o: int, v: int, seed: int = 0, naux: int | None = None,
                        device="cuda", row_chunk: int = 8192, with_vvvo: bool = True,
                        with_df: bool = False, b_scale: float = 1.0) -> dict:
    """Same recipe and the same random draws as ``make_problem`` (numpy
    PCG64 on the host), with the integral products formed in float64 on the
    GPU, for workloads whose (vv|vo) block does not fit host memory.
    ``with_df`` adds bvv, bvo and naux as in ``make_problem``;
    ``with_vvvo=False`` skips the (vv|vo) block; ``b_scale`` multiplies B."""
    import torch
    B, eps_o, eps_v, t1 = draw_factors(o, v, seed, naux, b_scale)
    naux = B.shape[0]
    Bd = torch.from_numpy(B).to(device)
    del B
    eps_o = torch.from_numpy(eps_o).to(device)
    eps_v = torch.from_numpy(eps_v).to(device)
    t1 = torch.from_numpy(np.ascontiguousarray(t1)).to(device)
    Bov = Bd[:, :o, o:].reshape(naux, o * v)
    Boo = Bd[:, :o, :o].reshape(naux, o * o)
    ovov = (Bov.t() @ Bov).reshape(o, v, o, v)
    ovov = (0.5 * (ovov + ovov.permute(2, 3, 0, 1))).contiguous()     # (ia|jb) = (jb|ia)
    ovoo = (Bov.t() @ Boo).reshape(o, v, o, o)
    ovoo = (0.5 * (ovoo + ovoo.permute(0, 1, 3, 2))).contiguous()     # (ia|jk) = (ia|kj)
    den = (eps_o[:, None, None, None] + eps_o[None, :, None, None]
           - eps_v[None, None, :, None] - eps_v[None, None, None, :])
    t2 = (ovov.permute(0, 2, 1, 3) / den).contiguous()
    out = dict(nocc=o, nvirt=v, eps_o=eps_o, eps_v=eps_v, t1=t1, t2=t2, ovoo=ovoo, ovov=ovov)
    if with_df:
        out["naux"] = naux
        out["bvv"] = Bd[:, o:, o:].permute(1, 2, 0).contiguous()
        out["bvo"] = Bd[:, o:, :o].permute(1, 2, 0).contiguous()
    if not with_vvvo:
        return out
    Bvv = Bd[:, o:, o:].reshape(naux, v * v)
    Bvo = Bd[:, o:, :o].reshape(naux, v * o).contiguous()
    del Bd
    vvvo = torch.empty((v * v, v * o), device=device, dtype=torch.float64)
    BvvT = Bvv.t()
    for r0 in range(0, v * v, row_chunk):
        r1 = min(v * v, r0 + row_chunk)
        torch.matmul(BvvT[r0:r1], Bvo, out=vvvo[r0:r1])
    del Bvv, BvvT, Bvo
    vvvo = vvvo.reshape(v, v, v, o)
    # (ab|ci) = (ba|ci): average each (a-block, b-block) pair with its mirror
    # once, so the symmetry is exact whatever the GEMM's summation order.
    step = 64
    for a0 in range(0, v, step):
        a1 = min(v, a0 + step)
        for b0 in range(a0, v, step):
            b1 = min(v, b0 + step)
            sym = 0.5 * (vvvo[a0:a1, b0:b1] + vvvo[b0:b1, a0:a1].transpose(0, 1))
            vvvo[a0:a1, b0:b1] = sym
            vvvo[b0:b1, a0:a1] = sym.transpose(0, 1)
    out["vvvo"] = vvvo
    return out




def make_mp2_problem(o: int, v: int, naux: int, seed: int = 0, device=None) -> dict:
    """RI-MP2 inputs: eps_o ~ U[-2.0, -0.3], eps_v ~ U[0.2, 5.0] and fitting
    coefficients c_ov[i][a][Q] ~ N(0, 0.1^2), drawn in that order from
    ``default_rng(seed)``, c_ov one occupied index at a time.  With ``device``
    the coefficients go to torch tensors on it, row by row, so that the host
    never holds all of them."""
    rng = np.random.default_rng(seed)
    eps_o = rng.uniform(-2.0, -0.3, size=o)
    eps_v = rng.uniform(0.2, 5.0, size=v)
    out = dict(nocc=o, nvirt=v, naux=naux)
    if device is None:
        c = np.empty((o, v, naux))
        for i in range(o):
            c[i] = rng.normal(0.0, 0.1, size=(v, naux))
        out.update(eps_o=eps_o, eps_v=eps_v, c_ov=c)
        return out
    import torch
    c = torch.empty((o, v, naux), dtype=torch.float64, device=device)
    for i in range(o):
        c[i].copy_(torch.from_numpy(rng.normal(0.0, 0.1, size=(v, naux))))
    out.update(eps_o=torch.from_numpy(eps_o).to(device), eps_v=torch.from_numpy(eps_v).to(device), c_ov=c)
    return out


def mp2_from_factors(o: int, v: int, seed: int = 0, naux: int | None = None) -> dict:
    """Tiny RI-MP2 problem whose coefficients are the ov block of the (T)
    recipe's symmetric factor B, c_ov[i][a][Q] = B^Q_{i,o+a}, together with
    the full ERI tensor built from all of B (for the spin-orbital check)."""
    B, eps_o, eps_v, _ = draw_factors(o, v, seed, naux)
    return dict(nocc=o, nvirt=v, naux=B.shape[0], eps_o=eps_o, eps_v=eps_v,
                c_ov=np.ascontiguousarray(B[:, :o, o:].transpose(1, 2, 0)), eri=full_eri(B))

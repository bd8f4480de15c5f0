"""Pins of the adjoint gradient against brute-force differentiation of the dense
assembled operator (tiny meshes, direct solves)."""
import numpy as np
import scipy.sparse as sp

import workload as wl
from oracle import adjoint
from oracle.sem import SemBox


def _dense_solver(box):
    def assemble(G):
        Ae = box.element_matrices(G)
        l2g = box.l2g.reshape(box.E, -1)
        A = np.zeros((box.n, box.n))
        for e in range(box.E):
            idx = l2g[e]
            keep = np.nonzero(idx >= 0)[0]
            A[np.ix_(idx[keep], idx[keep])] += Ae[e][np.ix_(keep, keep)]
        return A

    def solve(b, G=None):
        return np.linalg.solve(assemble(box.G if G is None else G), b)
    return solve


def test_gradient_matches_central_differences():
    box = SemBox(wl.deformed_box(2, 0.05), 3)
    solve = _dense_solver(box)
    xyz = box.coords()
    f = wl.manufactured_load(xyz)
    u_t = wl.target_field(xyz, seed=0)
    L0, u, dLdf, dLdG = adjoint.loss_and_grad(box, solve, f, u_t)
    B = box.mass()

    def loss(ff, GG):
        uu = solve(B * ff, GG)
        return float(np.dot(uu - u_t, uu - u_t))

    dirs = wl.gaussian_directions(6, (f.size, box.G.size), seed=1)
    h = 1e-6
    for vf, vG in dirs:
        vG = vG.reshape(box.G.shape)
        fd = (loss(f + h * vf, box.G + h * vG) - loss(f - h * vf, box.G - h * vG)) / (2 * h)
        an = float(np.dot(dLdf, vf) + np.sum(dLdG * vG))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * np.sqrt(np.sum(dLdG ** 2) + np.sum(dLdf ** 2)))


def test_single_factor_entries():
    # brute force on individual stored entries, including off-diagonal pairs stored once
    box = SemBox(wl.deformed_box(2, 0.08), 2)
    solve = _dense_solver(box)
    xyz = box.coords()
    f = wl.manufactured_load(xyz)
    u_t = wl.target_field(xyz, seed=2)
    _, _, _, dLdG = adjoint.loss_and_grad(box, solve, f, u_t)
    B = box.mass()
    rng = np.random.default_rng(3)
    for _ in range(12):
        idx = tuple(rng.integers(0, s) for s in box.G.shape)
        h = 1e-5 * abs(box.G[idx]) + 1e-9
        Gp, Gm = box.G.copy(), box.G.copy()
        Gp[idx] += h
        Gm[idx] -= h
        lp = np.sum((solve(B * f, Gp) - u_t) ** 2)
        lm = np.sum((solve(B * f, Gm) - u_t) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dLdG[idx]) <= 1e-5 * max(abs(fd), 1e-8)

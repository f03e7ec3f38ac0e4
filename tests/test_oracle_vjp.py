"""Pins for the oracle's vector-Jacobian product (CPU only).

The adjoint is not in the paper; it is derived from the energy and force
definitions (Sec. 2.2).  Pins:
  * central finite differences of the oracle's own forward (U, F);
  * autograd through an independent pure-PyTorch float64 implementation of
    the same energy and force (written directly from Eq. frbe);
  * translation invariance: sum_i dL/dr_i = 0;
  * charge homogeneity: U and F are quadratic in q, so
    sum_i q_i dL/dq_i = 2 (gU U + sum_i GF_i . F_i).
"""
import numpy as np
import torch

import rbe_inputs as ri
from oracle import sampler


def _loss(oracle_lib, s, x, y, z, q, m, w, gU, GF):
    F, U, _ = oracle_lib.force_energy(x, y, z, q, m, w, s.L)
    return gU * U + float(np.sum(GF * F))


def _setup(n=24, P=12, seed=4):
    s = ri.random_charges(n, 7.0, seed)
    m, S = sampler.sample_k(seed, 0, s.L, 0.5, P)
    w = np.full(P, S / P)
    GF = ri.gaussian_vectors(n, seed + 100)
    return s, m, w, 0.7, GF


def test_vjp_matches_finite_differences(oracle_lib):
    s, m, w, gU, GF = _setup()
    gr, gq = oracle_lib.vjp(s.x, s.y, s.z, s.q, m, w, s.L, gU, GF)
    h = 1e-5
    pos = [s.x, s.y, s.z]
    for i in range(s.n):
        for d in range(3):
            pp = [a.copy() for a in pos]
            pm = [a.copy() for a in pos]
            pp[d][i] += h
            pm[d][i] -= h
            fd = (_loss(oracle_lib, s, *pp, s.q, m, w, gU, GF) - _loss(oracle_lib, s, *pm, s.q, m, w, gU, GF)) / (2 * h)
            assert abs(fd - gr[d, i]) < 1e-6 * max(1.0, abs(fd)), (i, d, fd, gr[d, i])
        qp, qm = s.q.copy(), s.q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (_loss(oracle_lib, s, *pos, qp, m, w, gU, GF) - _loss(oracle_lib, s, *pos, qm, m, w, gU, GF)) / (2 * h)
        assert abs(fd - gq[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, gq[i])


def _torch_forward(x, y, z, q, m, w, L):
    """Independent float64 PyTorch RBE energy/force (Eq. frbe with per-k weights w)."""
    k = 2 * torch.pi * m.to(torch.float64) / L                 # (P, 3)
    r = torch.stack([x, y, z], dim=1)                          # (N, 3)
    th = r @ k.T                                               # (N, P)
    rho = torch.sum(q[:, None] * torch.exp(1j * th.to(torch.complex128)), dim=0)   # (P,)
    k2 = torch.sum(k * k, dim=1)
    c = w * 4 * torch.pi / (L ** 3 * k2)
    U = torch.sum(0.5 * c * torch.abs(rho) ** 2)
    im = torch.imag(torch.exp(-1j * th.to(torch.complex128)) * rho[None, :])   # (N, P)
    F = -q[:, None] * ((im * c[None, :]) @ k)                   # (N, 3)
    return U, F.T


def test_vjp_matches_torch_autograd(oracle_lib):
    s, m, w, gU, GF = _setup(n=64, P=16, seed=8)
    X = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (s.x, s.y, s.z, s.q)]
    U, F = _torch_forward(*X, torch.tensor(m), torch.tensor(w), s.L)
    Fo, Uo, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    assert abs(U.item() - Uo) < 1e-12 * abs(Uo)
    assert np.max(np.abs(F.detach().numpy() - Fo)) < 1e-12 * np.max(np.abs(Fo))
    lin = gU * U + torch.sum(torch.tensor(GF) * F)
    lin.backward()
    gr, gq = oracle_lib.vjp(s.x, s.y, s.z, s.q, m, w, s.L, gU, GF)
    ref_r = np.stack([X[0].grad.numpy(), X[1].grad.numpy(), X[2].grad.numpy()])
    assert np.max(np.abs(gr - ref_r)) < 1e-11 * np.max(np.abs(ref_r))
    assert np.max(np.abs(gq - X[3].grad.numpy())) < 1e-11 * np.max(np.abs(gq))


def test_vjp_identities(oracle_lib):
    s, m, w, gU, GF = _setup(n=200, P=30, seed=12)
    gr, gq = oracle_lib.vjp(s.x, s.y, s.z, s.q, m, w, s.L, gU, GF)
    F, U, _ = oracle_lib.force_energy(s.x, s.y, s.z, s.q, m, w, s.L)
    scale = np.max(np.abs(gr))
    assert np.max(np.abs(gr.sum(axis=1))) < 1e-12 * scale * s.n
    lhs = float(np.sum(s.q * gq))
    rhs = 2 * (gU * U + float(np.sum(GF * F)))
    assert abs(lhs - rhs) < 1e-11 * max(abs(rhs), 1.0)

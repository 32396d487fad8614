"""The Krylov-Schur eigensolver that computes the critical masses of the large
fields (tests/inputs/make_mcrit_gpu.py), run on the CPU against a dense
eigendecomposition of the oracle's Wilson operator on a small lattice."""
import importlib.util
import os

import numpy as np
import torch
from threadpoolctl import threadpool_limits

import synthetic
from oracle import wilson

_spec = importlib.util.spec_from_file_location(
    "make_mcrit_gpu", os.path.join(os.path.dirname(__file__), "inputs", "make_mcrit_gpu.py"))
mk = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mk)


def test_krylov_schur_finds_the_leftmost_eigenvalues_of_D0():
    dims = (2, 4, 2, 4)
    u = synthetic.gauge_field(dims, 0.45, seed=5)
    shape = (4, 2, 4, 2, 4, 3)
    n = int(np.prod(shape))
    dense = wilson.dense_D(u, 0.0)
    with threadpool_limits(1):  # a small dense problem; many BLAS threads only contend
        ev = np.linalg.eigvals(dense)
    ev = ev[np.argsort(ev.real)]

    def matvec(v):
        return torch.from_numpy(wilson.apply_D(u, v.numpy().reshape(shape), 0.0, -1.0).reshape(n))

    theta, res, V, C, nmv, cycles, done, hist = mk.krylov_schur_leftmost(
        matvec, n, torch.device("cpu"), 40, 12, 4, 1e-10, 500, 3, lambda s: None, 1e9)
    assert done
    assert np.allclose(theta[:4].real, ev[:4].real, atol=1e-9), (theta[:4], ev[:4])
    # the Ritz vector of the leftmost value is an eigenvector to the stated residual
    v = (torch.from_numpy(np.ascontiguousarray(C[:, 0])).unsqueeze(0) @ V[: C.shape[0]]).squeeze(0)
    r = matvec(v) - complex(theta[0]) * v
    assert float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(v)) < 1e-9


def test_chunked_basis_dots_equal_the_plain_product():
    g = torch.Generator().manual_seed(4)
    V = torch.randn(7, 1000, dtype=torch.complex128, generator=g)
    w = torch.randn(1000, dtype=torch.complex128, generator=g)
    for chunk in (64, 100, 1000, 4096):
        c = mk.basis_dots(V, w, chunk=chunk)
        assert float((c - V.conj() @ w).abs().max()) < 1e-12, chunk


def test_chunked_basis_combination_equals_the_plain_product():
    g = torch.Generator().manual_seed(5)
    V = torch.randn(6, 1000, dtype=torch.complex128, generator=g)
    c = torch.randn(6, dtype=torch.complex128, generator=g)
    for chunk in (64, 100, 1000, 4096):
        out = mk.basis_combine(V, c, chunk=chunk)
        assert float((out - c @ V).abs().max()) < 1e-12, chunk

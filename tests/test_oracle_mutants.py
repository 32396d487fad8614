"""Planted mistakes in the 4d oracle (on the CPU): each must fail at least one
pin of test_oracle_*.py, so that the pins, not the oracle's own formulas, carry
its correctness."""
import numpy as np
import pytest

from oracle import coarse, mg, transfer, wilson

import test_oracle_coarse as pins_coarse
import test_oracle_mg as pins_mg
import test_oracle_transfer as pins_transfer
import test_oracle_wilson as pins_wilson


def test_restriction_without_conjugation_is_caught(monkeypatch):
    def mutant(q, f, block):
        qb = transfer._split(q, block)
        fb = transfer._split(f, block)
        return np.einsum("kTtZzYyXxhn,...TtZzYyXxhn->...TZYXhk", qb, fb, optimize=True)
    monkeypatch.setattr(transfer, "restrict", mutant)
    with pytest.raises(AssertionError):
        pins_transfer.test_chirality_preserved_and_adjoint()


def test_exchanged_aggregate_faces_are_caught(monkeypatch):
    face_mask = coarse.face_mask
    monkeypatch.setattr(coarse, "face_mask", lambda site_shape, block, mu, sign: face_mask(site_shape, block, mu,
                                                                                           -sign))
    with pytest.raises(AssertionError):
        pins_coarse.test_stencil_matches_galerkin_definition((4, 4, 4, 4), (2, 2, 2, 2))


def test_mr_without_under_relaxation_is_caught(monkeypatch):
    mr = mg.mr
    monkeypatch.setattr(mg, "mr", lambda apply, x, r, iters, omega=0.8: mr(apply, x, r, iters, 1.0))
    with pytest.raises(AssertionError):
        pins_mg.test_mr_one_step_closed_form()


def test_ignored_time_boundary_sign_is_caught(monkeypatch):
    fwd, bwd = wilson.shift_fwd, wilson.shift_bwd
    monkeypatch.setattr(wilson, "shift_fwd", lambda f, mu, t_bc: fwd(f, mu, 1.0))
    monkeypatch.setattr(wilson, "shift_bwd", lambda f, mu, t_bc: bwd(f, mu, 1.0))
    with pytest.raises(AssertionError):
        pins_wilson.test_free_field_plane_wave_spectrum(-1.0)


def test_conjugated_step_size_is_caught(monkeypatch):
    # alpha = <r, D y> / <D y, D y> in place of <D y, r> / <D y, D y>
    dot = mg.dot
    calls = {"n": 0}

    def vcycle(self, l, r):
        apply = lambda f: self._apply(l, f)  # noqa: E731
        x = np.zeros_like(r)
        x, res = mg.mr(apply, x, r, self.nu_pre, self.omega)
        y = self.correction(l, res)
        dy = apply(y)
        a = dot(res, dy) / dot(dy, dy).real
        calls["n"] += 1
        x = x + a * y
        res = res - a * dy
        x, res = mg.mr(apply, x, res, self.nu_post, self.omega)
        return x
    monkeypatch.setattr(mg.Hierarchy, "vcycle", vcycle)
    with pytest.raises(AssertionError):
        pins_mg.test_alpha_step_leaves_a_residual_orthogonal_to_the_correction_image()
    assert calls["n"] >= 1


def test_flexible_cg_with_a_flipped_beta_is_caught(monkeypatch):
    from oracle import normal
    import test_oracle_normal as pins_normal

    def mutant(apply, b, tol, maxit=10000, precond=None, true_res=None, x0=None):
        m = precond if precond is not None else (lambda f: f.copy())
        x = np.zeros_like(b)
        r = b.copy()
        bn = mg.norm(b)
        info = {"iters": 0, "converged": False, "true_res": 1.0}
        p = q = None
        while info["iters"] < maxit:
            z = m(r)
            p = z if p is None else z + (mg.dot(q, z) / mg.dot(p, q)) * p  # sign of beta flipped
            q = apply(p)
            alpha = mg.dot(p, r) / mg.dot(p, q)
            x, r = x + alpha * p, r - alpha * q
            info["iters"] += 1
            if mg.norm(r) <= tol * bn:
                info["converged"] = True
                break
        info["true_res"] = mg.norm(b - apply(x)) / bn
        return x, info
    monkeypatch.setattr(normal, "fcg", mutant)
    with pytest.raises(AssertionError):
        pins_normal.test_fcg_is_cg_and_exact_with_the_inverse()


def test_probing_colours_that_alias_offsets_are_caught(monkeypatch):
    # colours repeating every 2 coarse sites: the +mu and -mu neighbours share a colour
    from oracle import normal
    import test_oracle_normal as pins_normal
    monkeypatch.setattr(normal, "colouring", lambda cdims: [2 if e % 2 == 0 else e for e in cdims])
    with pytest.raises(AssertionError):
        pins_normal.test_stencil_equals_the_literal_galerkin_map((12, 6, 6, 8), (4, 2, 2, 2), 2)

"""Planted mistakes in a copy of the oracle must be caught by its pins.

Each mutation is a plausible slip (a sign, a dropped term or square, a
conjugated form where the method needs the unconjugated one, a wrong rescale
at a seed switch).  The copy is executed from source in a fresh namespace on
the CPU; the real oracle module is untouched.
"""
import pathlib
import sys
import types

import numpy as np
import pytest

from oracle import dense_solve
from synth import bsr_to_scipy, make_problem

SRC = (pathlib.Path(__file__).resolve().parents[1] / "oracle" / "scocg.py").read_text()

MUTATIONS = {
    "shift_sign": ("alpha * (z[act] - z[s])", "alpha * (z[s] - z[act])"),
    "beta_not_squared": ("bk = ratio * ratio * beta", "bk = ratio * beta"),
    "alpha_unshifted": ("ak = ratio * alpha", "ak = (ratio / ratio) * alpha"),
    "conjugated_mu": ("mu = ps @ q", "mu = np.vdot(ps, q)"),
    "conjugated_gamma": ("gamma_new = rho @ r", "gamma_new = np.vdot(rho, r)"),
    "dropped_three_term": ("(beta_prev * alpha / alpha_prev) * (pi[act] - pi_old[act])",
                           "0.0 * (pi[act] - pi_old[act])"),
    "switch_old_rescale": ("pi_old[cand] = pi_old[cand] / co", "pi_old[cand] = pi_old[cand] / cn"),
    "switch_gamma": ("gamma = gamma / (cn * cn)", "gamma = gamma / cn"),
    "switch_beta_square": ("beta = (co / cn) ** 2 * beta", "beta = (co / cn) * beta"),
    "inner_unconjugated": ("a = rr / np.vdot(d, w).real", "a = rr / (d @ w).real"),
    "p_times_pi": ("r[:, None] / pin[None, :]", "r[:, None] * pin[None, :]"),
    "shift_H_sign": ("q = z[s] * (ps if S is None else S @ ps) - H @ ps",
                     "q = z[s] * (ps if S is None else S @ ps) + H @ ps"),
}


PROJ_MUTATIONS = {
    "proj_mu_sign": ("mu = r @ q - beta_prev * gamma / alpha_prev", "mu = r @ q + beta_prev * gamma / alpha_prev"),
    "proj_mu_conj": ("mu = r @ q - beta_prev", "mu = np.vdot(r, q) - beta_prev"),
    "proj_three_term": ("rho_new = (1.0 + c) * rho - alpha * q - c * rho_old",
                        "rho_new = rho - alpha * q"),
    "proj_old_rescale": ("rho, rho_old = rho / cn, rho_old / co", "rho, rho_old = rho / cn, rho_old / cn"),
    "proj_rows_update": ("pI[:, act] = r[rows][:, None] / pin[None, :]", "pI[:, act] = r[rows][:, None] * pin[None, :]"),
}


def _load(src):
    mod = types.ModuleType("oracle_mutant")
    sys.modules["oracle_mutant"] = mod          # dataclasses look the module up
    try:
        exec(compile(src, "oracle_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_mutant"]
    return mod


def _battery(mod):
    """Pins that a correct oracle passes: dense LU with and without S, with a
    forced seed switch.  Raises AssertionError on failure."""
    for s_scale, seed_key in ((None, (3, 1, 4)), (0.03, (2, 7, 1))):
        p = make_problem(lattice="sc", L=3, bdim=4, s_scale=s_scale, K=6, eta=0.1, nrhs=1,
                         seed_key=seed_key)
        H = bsr_to_scipy(p.H)
        S = bsr_to_scipy(p.S) if s_scale is not None else None
        b = np.zeros(p.M, dtype=np.complex128)
        b[int(p.rhs[0])] = 1.0
        with np.errstate(all="ignore"):
            res = mod.scocg(H, S, p.shifts, b, tol=1e-10, maxiter=2000, seed=0, inner_maxiter=200)
        assert len(res.seeds) > 1, "forced seed at the band edge must switch"
        assert np.all(res.status == 0), "not all shifts converged"
        for k, z in enumerate(p.shifts):
            xs = dense_solve(H, S, z, b)
            assert np.linalg.norm(res.x[:, k] - xs) <= 1e-7 * np.linalg.norm(xs)


def test_unmutated_copy_passes():
    _battery(_load(SRC))


def _mutate(fn_name, old, new):
    """Replace ``old`` by ``new`` inside the body of function ``fn_name`` only."""
    a = SRC.index(f"def {fn_name}(")
    b = SRC.find("\ndef ", a + 1)
    b = len(SRC) if b < 0 else b
    body = SRC[a:b]
    assert body.count(old) == 1, f"mutation anchor not found uniquely in {fn_name}: {old!r}"
    return SRC[:a] + body.replace(old, new) + SRC[b:]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    src = _mutate("inner_cg" if name == "inner_unconjugated" else "scocg", old, new)
    mod = _load(src)
    with pytest.raises((AssertionError, FloatingPointError, ZeroDivisionError, ValueError)):
        _battery(mod)


def _battery_projected(mod):
    for s_scale, seed_key in ((None, (3, 1, 4)), (0.03, (2, 7, 1))):
        p = make_problem(lattice="sc", L=3, bdim=4, s_scale=s_scale, K=6, eta=0.1, nrhs=1,
                         seed_key=seed_key)
        H = bsr_to_scipy(p.H)
        S = bsr_to_scipy(p.S) if s_scale is not None else None
        b = np.zeros(p.M, dtype=np.complex128)
        b[int(p.rhs[0])] = 1.0
        rows = p.outs(0)
        with np.errstate(all="ignore"):
            res = mod.scocg_projected(H, S, p.shifts, b, rows, tol=1e-10, maxiter=2000, seed=0,
                                      inner_maxiter=200)
        assert len(res.seeds) > 1, "forced seed at the band edge must switch"
        assert np.all(res.status == 0), "not all shifts converged"
        for k, z in enumerate(p.shifts):
            xs = dense_solve(H, S, z, b)[rows]
            assert np.linalg.norm(res.x[:, k] - xs) <= 1e-7 * np.linalg.norm(xs)


def test_unmutated_projected_passes():
    _battery_projected(_load(SRC))


@pytest.mark.parametrize("name", sorted(PROJ_MUTATIONS))
def test_projected_mutation_is_caught(name):
    old, new = PROJ_MUTATIONS[name]
    mod = _load(_mutate("scocg_projected", old, new))
    with pytest.raises((AssertionError, FloatingPointError, ZeroDivisionError, ValueError)):
        _battery_projected(mod)

"""Pins of the oracle's chemistry: stoichiometric invariants, detailed balance,
a forward-only closed form, the implicit substep's small-h consistency and its
fixed momentum and energy."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle import chem
from oracle.mesh import cartesian_mesh

T64 = torch.float64


def reacting_nodes(n=2000, seed=5, rho0=1e-3):
    """Random quiescent reacting nodes, T in [1000, 9000] K: state (1, 8, n)."""
    mech = di.air5_mechanism(42)
    rng = np.random.default_rng(seed)
    T = rng.uniform(1000.0, 9000.0, n)
    rho = rho0 * rng.uniform(0.9, 1.1, n)
    y = rng.uniform(0.05, 1.0, (5, n))
    y /= y.sum(0)
    rhos = rho * y
    U = np.zeros((1, 8, n))
    U[0, :5] = rhos
    U[0, 5] = rho * rng.uniform(-100, 100, n)
    U[0, 6] = rho * rng.uniform(-100, 100, n)
    U[0, 7] = (rhos * (mech["cv"][:, None] * T + mech["h0"][:, None])).sum(0) + \
        0.5 * (U[0, 5] ** 2 + U[0, 6] ** 2) / rho
    return mech, torch.tensor(U), torch.tensor(T)


def test_temperature_recovery():
    mech, U, T = reacting_nodes()
    rhos = [U[:, s] for s in range(5)]
    rho = sum(rhos)
    ke = 0.5 * (U[:, 5] ** 2 + U[:, 6] ** 2) / rho
    Trec = chem.temperature(mech, rhos, ke, U[:, 7])
    assert float((Trec[0] - T).abs().max() / T.max()) < 1e-13


def test_mass_and_atom_conservation():
    mech, U, _ = reacting_nodes()
    S = chem.source(mech, 2, U)
    w = [S[0, s] for s in range(5)]
    scale = max(float(x.abs().max()) for x in w)
    assert float(sum(w).abs().max()) <= 1e-15 * scale * 5
    # N atoms: N2 2, NO 1, N 1;  O atoms: O2 2, NO 1, O 1
    W = mech["W"]
    nN = 2 * w[0] / W[0] + w[2] / W[2] + w[3] / W[3]
    nO = 2 * w[1] / W[1] + w[2] / W[2] + w[4] / W[4]
    mscale = max(float((x / Wx).abs().max()) for x, Wx in zip(w, W))
    assert float(nN.abs().max()) <= 1e-15 * mscale * 5
    assert float(nO.abs().max()) <= 1e-15 * mscale * 5
    # momentum and energy rows carry no source
    assert float(S[0, 5:].abs().max()) == 0.0


def single_reaction(mech, r, reversible):
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in mech.items()}
    for q in range(5):
        if q != r:
            m["A_f"][q] = 0.0
            m["A_b"][q] = 0.0
    m["reversible"] = np.array([1 if (q == r and reversible) else 0 for q in range(5)], dtype=np.int32)
    return m


def test_forward_only_closed_form():
    """N2 + M -> 2N + M alone: wdot_N2 = -kappa_r W_N2 k_f [N2][M],
    wdot_N = +2 kappa_r W_N k_f [N2][M], [M] = sum of all concentrations."""
    mech, U, T = reacting_nodes(200)
    m = single_reaction(mech, 0, reversible=False)
    S = chem.source(m, 2, U)
    X = [1e-6 * U[0, s] / m["W"][s] for s in range(5)]
    kf = m["A_f"][0] * np.power(T.numpy(), m["beta_f"][0]) * np.exp(-m["theta_f"][0] / T.numpy())
    rate = kf * X[0].numpy() * sum(x.numpy() for x in X)
    np.testing.assert_allclose(S[0, 0].numpy(), -1e6 * m["W"][0] * rate, rtol=1e-12)
    np.testing.assert_allclose(S[0, 3].numpy(), 2e6 * m["W"][3] * rate, rtol=1e-12)
    for s in (1, 2, 4):
        assert float(S[0, s].abs().max()) == 0.0


def test_detailed_balance_zero_rate():
    """N2 + O <=> NO + N with [NO] chosen so that k_f [N2][O] = k_b [NO][N]."""
    mech, U, T = reacting_nodes(100)
    m = single_reaction(mech, 3, reversible=True)
    Tn = T.numpy()
    kf = m["A_f"][3] * Tn ** m["beta_f"][3] * np.exp(-m["theta_f"][3] / Tn)
    kb = m["A_b"][3] * Tn ** m["beta_b"][3] * np.exp(-m["theta_b"][3] / Tn)
    U = U.clone()
    X = [1e-6 * U[0, s].numpy() / m["W"][s] for s in range(5)]
    XNO = kf * X[0] * X[4] / (kb * X[3])
    U[0, 2] = torch.tensor(XNO * m["W"][2] / 1e-6)
    # keep T fixed by recomputing E for the new composition
    rhos = U[0, :5].numpy()
    rho = rhos.sum(0)
    U[0, 7] = torch.tensor((rhos * (m["cv"][:, None] * Tn + m["h0"][:, None])).sum(0)
                           + 0.5 * (U[0, 5].numpy() ** 2 + U[0, 6].numpy() ** 2) / rho)
    S = chem.source(m, 2, U)
    # each term of the net rate is ~ kf [N2][O]; the difference must cancel
    Rterm = 1e6 * kf * X[0] * X[4] * m["W"][2]
    assert float((S[0, 2].abs() / torch.tensor(Rterm)).max()) < 1e-12


def test_implicit_substep_small_h_consistency():
    """BE: Y* = Y + h S(Y) + O(h^2): the defect quarters when h halves (h far
    below the fastest chemical time of the mechanism, the backward rates
    reaching 1e22 in CGS units)."""
    mech, U, _ = reacting_nodes(300, rho0=1e-3)
    S = chem.source(mech, 2, U)
    defects = []
    for h in (1e-14, 5e-15, 2.5e-15):
        Un, st = chem.implicit_substep(mech, 2, U, h)
        assert st["unconverged"] == 0
        defects.append(float((Un[:, :5] - U[:, :5] - h * S[:, :5]).abs().max()))
    r = [defects[i] / defects[i + 1] for i in range(2)]
    assert all(3.0 < x < 5.0 for x in r), r


def test_implicit_substep_workload():
    """On a coarse copy of the reacting workload (surveyed stiffness: rho about
    0.1 kg/m^3, backward rates over the forward range) with h = dt/2 at CFL
    0.5: Newton converges everywhere, momentum and energy are untouched, the
    species sum is kept to round-off and the converged residual is small."""
    p = di.PRESETS["air5_2d"]
    mech = di.preset_mechanism(p)
    m = cartesian_mesh(2, 3, (16, 16), p["lo"], p["hi"], (6, 6), (10, 10))
    U = torch.tensor(di.reacting_state(m.coords(), p["lo"], p["hi"], mech, rho0=p["rho0"]))[None]
    h = 2.1e-7
    Un, st = chem.implicit_substep(mech, 2, U, h)
    assert st["unconverged"] == 0
    assert torch.equal(Un[:, 5:], U[:, 5:])
    rho0 = U[:, :5].sum(1)
    rho1 = Un[:, :5].sum(1)
    assert float(((rho1 - rho0) / rho0).abs().max()) < 1e-13
    # residual of the backward-Euler equation at the returned state
    S = chem.source(mech, 2, Un)
    res = (Un[:, :5] - U[:, :5] - h * S[:, :5]).abs().amax(dim=1) / rho0
    hs = (h * S[:, :5]).abs().amax(dim=1) / rho0
    assert float((res / torch.clamp(hs, min=1.0)).max()) < 1e-9


# atoms of N and O per unit mass of each species (N2, O2, NO, N, O)
def atoms(mech, Y):
    A = torch.tensor([[2.0, 0.0, 1.0, 1.0, 0.0], [0.0, 2.0, 1.0, 0.0, 1.0]], dtype=torch.float64)
    return (A / torch.tensor(mech["W"])[None]) @ Y


@pytest.mark.slow
def test_implicit_substep_full_workload_stiff():
    """The full reacting workload (77,824 nodes) at h = dt/2: the plain
    Newton iteration from Y^n is drawn to a spurious corner on a few per
    cent of the nodes (a species at zero, residual of order h |S|); with the
    continuation in h every node reaches the root: residual at the round-off
    level, mass and N and O atoms conserved."""
    from oracle.dgsem import Operator
    from oracle.physics import ReactingEuler
    from oracle.timestep import dt_cfl
    p = di.PRESETS["air5_2d"]
    mech = di.preset_mechanism(p)
    m = cartesian_mesh(2, 3, p["nel"], p["lo"], p["hi"], p["patch_lo"], p["patch_hi"])
    U = torch.tensor(di.reacting_state(m.coords(), p["lo"], p["hi"], mech, rho0=p["rho0"]))[None]
    h = 0.5 * dt_cfl(Operator(m, ReactingEuler(2, mech)), U, p["cfl"])
    Un, st = chem.implicit_substep(mech, 2, U, h)
    assert st["unconverged"] == 0
    assert st["continued"] > 0.005 * U[0, 0].numel()
    Y0 = U[0, :5].reshape(5, -1)
    Y1 = Un[0, :5].reshape(5, -1)
    rho = Y0.sum(0)
    R = Y1 - Y0 - h * chem.source(mech, 2, Un)[0, :5].reshape(5, -1)
    assert float((R.abs().amax(0) / rho).max()) < 1e-12
    assert float((atoms(mech, Y1 - Y0).abs().amax(0) / (atoms(mech, Y0).abs().amax(0))).max()) < 1e-13
    assert float(((Y1.sum(0) - rho) / rho).abs().max()) < 1e-13
    # without the continuation (a mistake planted in the algorithm) the same
    # nodes are left unconverged
    _, st0 = chem.implicit_substep(mech, 2, U, h, levels=-1)
    assert st0["unconverged"] > 0.005 * U[0, 0].numel()


def test_implicit_substep_small_h_consistency_stiff():
    """BE at the surveyed density: Y* = Y + h S(Y) + O(h^2) for small h."""
    mech = di.preset_mechanism(di.PRESETS["air5_2d"])
    _, U, _ = reacting_nodes(300, rho0=0.1)
    U = U.clone()
    S = chem.source(mech, 2, U)
    defects = []
    for h in (1e-16, 5e-17, 2.5e-17):
        Un, st = chem.implicit_substep(mech, 2, U, h)
        assert st["unconverged"] == 0
        defects.append(float((Un[:, :5] - U[:, :5] - h * S[:, :5]).abs().max()))
    r = [defects[i] / defects[i + 1] for i in range(2)]
    assert all(3.0 < x < 5.0 for x in r), r

"""Pins of the oracle's two-temperature model against what the physics and the
mathematics fix: the harmonic-oscillator energy's limits, the T_v inversion,
reduction of the two-temperature rates to the one-temperature ones at
T_v = T, mass and atom conservation, the Landau-Teller term's zero and sign,
the 1/p scaling of the relaxation time, the implicit substep's consistency,
its relaxation to T_v = T and its invariants, and free stream and
conservation of the two-temperature operator (E_v column included)."""

import copy
import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.chem import wdot
from oracle.dgsem import Operator
from oracle.mesh import cartesian_mesh
from oracle.twotemp import (ReactingEuler2T, e_vib, implicit_substep, q_vt, source, t_vib, tau_vt, vib_energy,
                            wdot_2t)
from oracle.timestep import integrals

MECH = di.preset_mechanism(di.PRESETS["air5_2t_2d"])
VIB = di.air5_vibration(MECH)
ATOMS = np.array([[2, 0], [0, 2], [1, 1], [1, 0], [0, 1]])    # (N, O) atoms per species


def random_node_state(n, seed, T_range=(2000.0, 9000.0)):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5e-3, 2e-3, n)
    y = rng.uniform(0.05, 1.0, (5, n))
    y /= y.sum(axis=0)
    rhos = [torch.tensor(rho * y[s]) for s in range(5)]
    T = torch.tensor(rng.uniform(*T_range, n))
    Tv = torch.tensor(rng.uniform(*T_range, n))
    return rhos, T, Tv


def test_vibrational_energy_limits():
    th, R = VIB["theta_v"][0], MECH["R"][0]
    T = torch.tensor([100.0 * th, 1000.0 * th], dtype=torch.float64)
    x = th / T
    series = R * T * (1 - x / 2 + x ** 2 / 12 - x ** 4 / 720)
    assert float(((e_vib(th, R, T) - series) / series).abs().max()) < 1e-13
    T = torch.tensor([th / 30.0, th / 60.0], dtype=torch.float64)
    low = R * th * torch.exp(-th / T)
    assert float(((e_vib(th, R, T) - low) / low).abs().max()) < 1e-12
    assert float(e_vib(0.0, MECH["R"][3], T).abs().max()) == 0.0


def test_t_vib_inverts_vib_energy():
    rhos, _, Tv = random_node_state(500, 1, T_range=(300.0, 30000.0))
    Ev = vib_energy(MECH, VIB, rhos, Tv)
    back = t_vib(MECH, VIB, rhos, Ev)
    assert float(((back - Tv) / Tv).abs().max()) < 1e-13


def test_rates_reduce_to_one_temperature_at_equilibrium():
    rhos, T, _ = random_node_state(300, 2)
    w2 = wdot_2t(MECH, VIB, rhos, T, T.clone())
    w1 = wdot(MECH, rhos, T)
    for s in range(5):
        assert torch.allclose(w2[s], w1[s], rtol=1e-13, atol=1e-300)
    # and differ once T_v != T (only the dissociations change)
    w3 = wdot_2t(MECH, VIB, rhos, T, 0.7 * T)
    assert not torch.allclose(w3[0], w1[0], rtol=1e-6)


def test_mass_and_atom_conservation():
    rhos, T, Tv = random_node_state(400, 3)
    w = torch.stack(wdot_2t(MECH, VIB, rhos, T, Tv))
    scale = w.abs().sum(dim=0)
    assert float((w.sum(dim=0).abs() / scale).max()) < 1e-13
    moles = w / torch.tensor(MECH["W"])[:, None]
    for a in range(2):
        atoms = (torch.tensor(ATOMS[:, a], dtype=torch.float64)[:, None] * moles).sum(dim=0)
        assert float((atoms.abs() / (moles.abs().sum(dim=0))).max()) < 1e-13


def test_landau_teller_zero_and_sign():
    rhos, T, Tv = random_node_state(400, 4)
    p = T * sum(rhos[s] * MECH["R"][s] for s in range(5))
    assert float(q_vt(MECH, VIB, rhos, T, T.clone(), p).abs().max()) == 0.0
    q = q_vt(MECH, VIB, rhos, T, Tv, p)
    assert bool(((q > 0) == (Tv < T)).all())


def test_relaxation_time_scales_as_inverse_pressure():
    rhos, T, _ = random_node_state(200, 5)
    p = T * sum(rhos[s] * MECH["R"][s] for s in range(5))
    t1 = tau_vt(MECH, VIB, rhos, T, p)
    t2 = tau_vt(MECH, VIB, rhos, T, 2.0 * p)
    for s in range(3):
        assert torch.allclose(t2[s], 0.5 * t1[s], rtol=1e-13, atol=0)
        assert bool((t1[s] > 0).all())
    assert float(t1[3].abs().max()) == 0.0


def node_state(n, seed, u0=0.0):
    """(1, nv, n) two-temperature states from the seeded generator's recipe
    on random nodes."""
    m = cartesian_mesh(2, 3, (2, 2), (-1, -1), (1, 1))
    X = m.coords().reshape(2, -1)[:, :n]
    return torch.tensor(di.reacting2t_state(X, (-1, -1), (1, 1), MECH, VIB, u0=u0))[None]


def test_source_rows():
    phys = ReactingEuler2T(2, MECH, VIB)
    U = node_state(64, 0, u0=300.0)
    S = source(phys, U)
    assert float(S[:, 5:8].abs().max()) == 0.0               # momentum and E rows
    frozen = copy.deepcopy(MECH)
    frozen["A_f"] = np.zeros(5)
    frozen["A_b"] = np.zeros(5)
    Sf = source(ReactingEuler2T(2, frozen, VIB), U)
    assert float(Sf[:, :5].abs().max()) == 0.0
    assert float(Sf[:, 8].abs().max()) > 0.0


def test_implicit_substep_consistency_and_invariants():
    phys = ReactingEuler2T(2, MECH, VIB)
    U = node_state(64, 0, u0=300.0)
    S = source(phys, U)
    errs = []
    # the seeded rates are stiff at 9000 K (timescales near 1e-10 s): the
    # asymptotic regime of the O(h^2) difference starts below h = 1e-12
    for h in (2e-13, 1e-13):
        Un, st = implicit_substep(phys, U, h)
        assert st["unconverged"] == 0
        errs.append(float(((Un - U - h * S)[:, [0, 1, 2, 3, 4, 8]]).abs().max()))
    assert 3.0 < errs[0] / errs[1] < 5.0, errs                # backward Euler: O(h^2) from forward Euler
    Un, st = implicit_substep(phys, U, 1e-6)
    assert torch.equal(Un[:, 5:8], U[:, 5:8])                  # momentum and E untouched
    assert torch.allclose(Un[:, :5].sum(1), U[:, :5].sum(1), rtol=1e-13, atol=0)
    dm = (Un[:, :5] - U[:, :5])[0] / torch.tensor(MECH["W"])[:, None]
    for a in range(2):
        atoms = (torch.tensor(ATOMS[:, a], dtype=torch.float64)[:, None] * dm).sum(0)
        assert float(atoms.abs().max()) < 1e-12 * float(U[:, :5].abs().max())


def test_pure_vibrational_relaxation_reaches_equilibrium():
    frozen = copy.deepcopy(MECH)
    frozen["A_f"] = np.zeros(5)
    frozen["A_b"] = np.zeros(5)
    phys = ReactingEuler2T(2, frozen, VIB)
    U = node_state(64, 0)
    Un, st = implicit_substep(phys, U, 1.0e4)                  # h >> tau
    assert st["unconverged"] == 0
    P = phys.prims(Un)
    rhos = P["rhos"]
    Tv = t_vib(frozen, VIB, rhos, Un[:, 8])
    assert float(((Tv - P["T"]) / P["T"]).abs().max()) < 1e-6
    assert torch.equal(Un[:, :5], U[:, :5])


@pytest.mark.parametrize("patch", [None, ((1, 1), (3, 3))])
def test_operator_free_stream_and_conservation(patch):
    m = cartesian_mesh(2, 3, (5, 4), (-1, -1), (1, 1), *(patch or (None, None)))
    phys = ReactingEuler2T(2, MECH, VIB)
    op = Operator(m, phys)
    U = torch.tensor(di.reacting2t_state(m.coords(), (-1, -1), (1, 1), MECH, VIB, u0=300.0))[None]
    c = U.mean(dim=tuple(range(2, U.dim())), keepdim=True).expand_as(U).clone()
    dc = op.rhs(c)
    # rounding in the flux sums is relative to the fluxes, not to the state
    P = phys.prims(c)
    Fs = torch.stack([phys.flux(c, l, P).abs().amax(dim=(0, 2, 3, 4)) for l in range(2)]).amax(dim=0)
    Fs = Fs * float(op.D.abs().sum(1).max()) * 2.0 / m.hmin()
    assert float((dc.abs().amax(dim=(0, 2, 3, 4)) / Fs.clamp_min(1e-300)).max()) < 1e-13
    dU = op.rhs(U)
    I = integrals(op, dU, with_ke=False)[:, :-1]
    Wt = op.J.reshape(-1, 1, 1)
    from oracle.timestep import tensor_weights
    scale = ((Wt * tensor_weights(op)) * dU.abs()).sum(dim=(2, 3, 4)).numpy()
    assert np.abs(I / scale).max() < 1e-12


def test_chemistry_leaves_t_vib_unchanged_at_equilibrium():
    """With T_v = T the Landau-Teller term vanishes and the E_v row is the
    vibrational energy carried by the molecules made or destroyed: a small
    step along the source keeps T_v fixed (checked through the independent
    inversion), which fails if the sum wdot_s e_v,s(T_v) is dropped or
    mis-weighted."""
    rhos, T, _ = random_node_state(200, 6, T_range=(4000.0, 8000.0))
    p = T * sum(rhos[s] * MECH["R"][s] for s in range(5))
    w = wdot_2t(MECH, VIB, rhos, T, T)
    Ev = vib_energy(MECH, VIB, rhos, T)
    from oracle.twotemp import source_terms
    _, sev = source_terms(MECH, VIB, rhos, T, T.clone())
    # delta small against the fastest species change at these temperatures
    delta = 1e-3 * float(min((rhos[s] / w[s].abs().clamp_min(1e-300)).min() for s in range(5)))
    rp = [rhos[s] + delta * w[s] for s in range(5)]
    Tv = t_vib(MECH, VIB, rp, Ev + delta * sev)
    assert float(((Tv - T) / T).abs().max()) < 1e-9
    assert float(sev.abs().max()) > 0.0


def test_exchange_reactions_take_the_translational_temperature():
    only_exchange = copy.deepcopy(MECH)
    only_exchange["A_f"] = np.array(MECH["A_f"]) * np.array([0, 0, 0, 1, 1])
    only_exchange["A_b"] = np.array(MECH["A_b"]) * np.array([0, 0, 0, 1, 1])
    rhos, T, Tv = random_node_state(300, 7)
    w2 = wdot_2t(only_exchange, VIB, rhos, T, Tv)
    w1 = wdot(only_exchange, rhos, T)
    for s in range(5):
        assert torch.allclose(w2[s], w1[s], rtol=1e-13, atol=1e-300)


def test_operator_advects_vibrational_energy():
    """Uniform velocity, temperature and composition with a sinusoidal E_v
    (pressure uniform): the E_v row of L(U) is -u . grad E_v, the other rows
    follow E's advection; error falls with resolution."""
    errs = []
    for nel in (4, 8):
        m = cartesian_mesh(2, 3, (nel, nel), (0, 0), (1, 1))
        phys = ReactingEuler2T(2, MECH, VIB)
        op = Operator(m, phys)
        x, y = m.coords()
        x, y = torch.tensor(x), torch.tensor(y)
        rho, T, u = 1e-3, 5000.0, (120.0, -80.0)
        yfr = torch.tensor([0.4, 0.2, 0.1, 0.2, 0.1], dtype=torch.float64)
        rhos = [rho * yfr[s] * torch.ones_like(x) for s in range(5)]
        Ev = 200.0 + 50.0 * torch.sin(2 * math.pi * x) * torch.cos(2 * math.pi * y)
        E = sum(rhos[s] * (MECH["cv"][s] * T + MECH["h0"][s]) for s in range(5)) + Ev + 0.5 * rho * (u[0] ** 2 + u[1] ** 2)
        U = torch.stack(rhos + [rho * u[0] * torch.ones_like(x), rho * u[1] * torch.ones_like(x), E, Ev])[None]
        dEv = 50.0 * 2 * math.pi * (torch.cos(2 * math.pi * x) * torch.cos(2 * math.pi * y) * u[0]
                                    - torch.sin(2 * math.pi * x) * torch.sin(2 * math.pi * y) * u[1])
        dU = op.rhs(U)
        errs.append(float((dU[0, 8] + dEv).abs().max() / dEv.abs().max()))
        assert float(dU[0, :5].abs().max()) < 1e-9 * rho * 300.0
    assert errs[1] < 0.25 * errs[0] and errs[1] < 1e-2, errs


def test_park_limit_at_high_temperature():
    """Far above the vibrational temperatures Park's limiting time dominates
    and scales as T^2.5 at fixed pressure (sigma_v ~ T^-2, cbar ~ T^0.5,
    n ~ 1/T)."""
    rhos, _, _ = random_node_state(50, 8)
    T1 = torch.full_like(rhos[0], 5.0e4)
    T2 = torch.full_like(rhos[0], 1.0e5)
    p = torch.full_like(rhos[0], 1.0e4)
    t1, t2 = tau_vt(MECH, VIB, rhos, T1, p), tau_vt(MECH, VIB, rhos, T2, p)
    for s in range(3):
        assert torch.allclose(t2[s] / t1[s], torch.full_like(T1, 2.0 ** 2.5), rtol=2e-2)


def test_closure_recovers_the_generating_temperature():
    """The state generator builds E from a temperature field T0 + dT g
    (seed 10) with E_v on top; the closure must return that T (E_v is not
    translational energy)."""
    m = cartesian_mesh(2, 3, (3, 3), (-1, -1), (1, 1))
    X = m.coords()
    U = torch.tensor(di.reacting2t_state(X, (-1, -1), (1, 1), MECH, VIB, u0=250.0))[None]
    T = torch.tensor(5000.0 + 4000.0 * di.fourier_field(X, (-1, -1), (1, 1), seed=10))
    P = ReactingEuler2T(2, MECH, VIB).prims(U)
    assert float(((P["T"][0] - T) / T).abs().max()) < 1e-12

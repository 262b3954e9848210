"""Shared helpers of the GPU parity tests: build an oracle operator and a
library context for the same problem, move states between them, and the
norm-wise error used throughout (per variable, ||x - y||_inf / ||y||_inf)."""

import numpy as np
import torch

import dginputs as di
from oracle.dgsem import Operator
from oracle.split import SplitOperator
from oracle.mesh import cartesian_mesh
from oracle.physics import Euler, ReactingEuler


def make_pair(dim, N, nel, lo, hi, physics="euler", precision="f64", batch=1, patch=None,
              mu=0.0, prandtl=0.72, mech=None, volume="standard", vib=None):
    from paper_2605_26388_amd import Solver
    plo, phi = patch if patch else (None, None)
    mesh = cartesian_mesh(dim, N, nel, lo, hi, plo, phi)
    viscous = None
    if physics == "reacting":
        phys = ReactingEuler(dim, mech)
    elif physics == "reacting_2t":
        from oracle.twotemp import ReactingEuler2T
        phys = ReactingEuler2T(dim, mech, vib)
    else:
        phys = Euler(dim)
        if physics == "navier_stokes":
            viscous = dict(mu=mu, prandtl=prandtl, gamma=1.4)
    if volume == "split":
        op = SplitOperator(mesh, phys, viscous=viscous)
    else:
        op = Operator(mesh, phys, viscous=viscous)
    s = Solver(dim, N, nel, lo, hi, physics=physics, precision=precision, batch=batch,
               patch_lo=plo, patch_hi=phi, mu=mu, prandtl=prandtl, mech=mech, volume=volume, vib=vib)
    assert s.E == mesh.E
    return op, s


def to_gpu(s, U):
    """Oracle layout (B, nv, E, n..n) float64 -> library tensor."""
    return U.reshape(s.shape).to(device=s.device, dtype=s.dtype).contiguous()


def from_gpu(op, X):
    return X.detach().to("cpu", torch.float64).reshape((X.shape[0], X.shape[1], X.shape[2]) + (op.n,) * op.dim)


def rel_err(got, ref):
    """max over variables of ||got_v - ref_v||_inf / ||ref_v||_inf."""
    B, nv = ref.shape[:2]
    g = got.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    r = ref.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    num = (g - r).abs().amax(dim=1)
    den = r.abs().amax(dim=1).clamp_min(1e-300)
    return float((num / den).max())


def random_euler_state(op, seed, B=1):
    rng = np.random.default_rng(seed)
    shape = (B, op.mesh.E) + (op.n,) * op.dim
    rho = rng.uniform(0.5, 1.5, shape)
    vel = [rng.uniform(-0.5, 0.5, shape) for _ in range(op.dim)]
    p = rng.uniform(0.5, 1.5, shape)
    return torch.tensor(np.stack([di.conserved_from_primitive(rho[b], [v[b] for v in vel], p[b], 1.4)
                                  for b in range(B)]))


def smooth_euler_state(op, B=1):
    X = op.mesh.coords()
    base = di.random_euler(X, op.mesh.lo, op.mesh.hi)
    if B == 1:
        return torch.tensor(base)[None]
    return torch.tensor(np.stack([di.perturb_density(base, b) for b in range(B)]))


def flux_scale(op, U):
    """Per-variable size of the terms a right-hand side is assembled from:
    (2/h_min) ||D||_inf max_l ||F_l,v||_inf.  Rounding in a sweep of D is
    relative to this, not to the (possibly much smaller) result; e.g. at low
    Mach number the momentum flux carries the large mean pressure."""
    P = op.phys.prims(U)
    Dn = float(op.D.abs().sum(1).max())
    s = None
    for l in range(op.dim):
        F = op.phys.flux(U, l, P).abs()
        m = F.transpose(0, 1).reshape(F.shape[1], -1).amax(dim=1)
        s = m if s is None else torch.maximum(s, m)
    return s * Dn * 2.0 / op.mesh.hmin()


def rel_err_floor(got, ref, floor):
    """max over variables of ||got_v - ref_v||_inf / max(||ref_v||_inf, floor_v)."""
    B, nv = ref.shape[:2]
    g = got.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    r = ref.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    num = (g - r).abs().amax(dim=1)
    den = torch.maximum(r.abs().amax(dim=1), floor.to(r.dtype))
    return float((num / den).max())


def mirror(U, nel, dirs, mom=1):
    """Mirror image of a state on a lexicographic (x fastest) element grid:
    reverse the element and node order along each direction in `dirs` and
    negate those momentum components.  L(mirror(U)) = mirror(L(U)) in exact
    arithmetic whenever the mesh is invariant under the mirror (any periodic
    Cartesian box for one direction; the warped meshes for pairs of
    directions, a half turn), while every derivative sum and every interface
    flux is evaluated in reversed order."""
    B, nv, E = U.shape[:3]
    dim = len(nel)
    n = U.shape[-1]
    X = U.reshape((B, nv) + tuple(reversed(nel)) + (n,) * dim).clone()
    for l in dirs:
        X = X.flip(2 + dim - 1 - l).flip(2 + dim + dim - 1 - l)
        X[:, mom + l] = -X[:, mom + l]
    return X.reshape(U.shape)


def cycle(U, nel, mom=1):
    """Relabel the axes of a 3-D state on a cube of equal element counts,
    (x, y, z) -> (y, z, x): the arrays are transposed and the momentum
    components permuted with them.  L(cycle(U)) = cycle(L(U)) in exact
    arithmetic; the derivative sums then run along other memory axes."""
    assert len(nel) == 3 and nel[0] == nel[1] == nel[2]
    B, nv, E = U.shape[:3]
    n = U.shape[-1]
    X = U.reshape((B, nv) + tuple(reversed(nel)) + (n,) * 3)
    X = X.permute(0, 1, 4, 2, 3, 7, 5, 6)
    idx = list(range(nv))
    idx[mom:mom + 3] = [mom + 1, mom + 2, mom]
    return X[:, idx].reshape(U.shape).contiguous()


def rounding_spread(rhs, U, nel, mirrors, cycles=False):
    """Per-variable rounding spread of the oracle's own FP64 arithmetic at U:
    the largest |L(U) - mirror(L(mirror(U)))| over the mirror images in
    `mirrors` (and, with cycles=True on a cube, over the two cyclic
    relabellings of the axes).  The mirrored evaluation sees the same input bits (so the same
    interface jumps) but forms every derivative sum and every interface flux
    in reversed order: the difference is what two correct FP64 evaluations of
    L differ by at this state, the floor below which a parity comparison
    cannot see.  Returns (L(U), spread)."""
    R = rhs(U)
    B, nv = R.shape[:2]
    s = torch.zeros(nv, dtype=torch.float64)
    cands = [lambda X, d=d: mirror(X, nel, d) for d in mirrors]
    inv = [lambda X, d=d: mirror(X, nel, d) for d in mirrors]
    if cycles:
        cands += [lambda X: cycle(X, nel), lambda X: cycle(cycle(X, nel), nel)]
        inv += [lambda X: cycle(cycle(X, nel), nel), lambda X: cycle(X, nel)]
    for f, g in zip(cands, inv):
        C = g(rhs(f(U)))
        s = torch.maximum(s, (C - R).reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1).abs().amax(dim=1))
    return R, s


# Parity bound where cancellation sets the floor: per variable
#   ||got_v - ref_v||_inf <= max(1e-12 ||ref_v||_inf, SPREAD_FACTOR * spread_v).
# The library forms reciprocals to within 11 units in the last place (the
# oracle divides, 0.5) and sums in a different order, so its own rounding
# error can be up to about 10 times the oracle's; the difference of the two is
# then within about 11 spreads, and the factor 16 leaves headroom on that.
SPREAD_FACTOR = 16.0


def spread_err(got, ref, spread, rel=1e-12):
    """max over variables of ||got_v - ref_v||_inf / max(rel ||ref_v||_inf,
    SPREAD_FACTOR spread_v): below 1 passes."""
    B, nv = ref.shape[:2]
    g = got.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    r = ref.reshape(B, nv, -1).transpose(0, 1).reshape(nv, -1)
    num = (g - r).abs().amax(dim=1)
    den = torch.maximum(rel * r.abs().amax(dim=1), SPREAD_FACTOR * spread.to(r.dtype)).clamp_min(1e-300)
    return float((num / den).max())

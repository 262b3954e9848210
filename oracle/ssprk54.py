"""Five-stage, fourth-order SSP Runge-Kutta method and the per-stage
positivity floor (SSP-RK Time Discretization appendix; the floor is named in
the configurations of the paper's Euler and Navier-Stokes cases) -- test
infrastructure, as the rest of the oracle.

The appendix writes an s-stage SSP method in Shu-Osher form,
    U^(0) = U^n,  U^(i) = sum_{k<i} [alpha_ik U^(k) + dt beta_ik L(U^(k))],
    U^(n+1) = U^(s),
with alpha_ik, beta_ik >= 0 and sum_k alpha_ik = 1, and names the method of
Spiteri and Ruuth with SSP coefficient about 1.508, without printing its
coefficients.  The table below holds that method's published Shu-Osher
coefficients (to 15 digits).  They are pinned in the tests by what fixes
them mathematically: the eight fourth-order conditions of the equivalent
Butcher tableau, the row sums of alpha, and the SSP coefficient
min alpha_ik / beta_ik = 1.508.

Positivity floor (reading: the paper gives the bounds, rho >= rho_min and
p >= p_min applied after every stage, not the operation): node by node,
    rho <- max(rho, rho_min)                      (momentum unchanged),
    E   <- max(E, p_min/(gamma-1) + |m|^2/(2 rho)) (with that rho),
i.e. density clipped, then the total energy raised just enough that the
pressure at that density and momentum is p_min.  It acts on nothing else.
"""

import torch

# nonzero Shu-Osher coefficients (i, k): stage i takes stage k
ALPHA = {
    (1, 0): 1.0,
    (2, 0): 0.444370493651235, (2, 1): 0.555629506348765,
    (3, 0): 0.620101851488403, (3, 2): 0.379898148511597,
    (4, 0): 0.178079954393132, (4, 3): 0.821920045606868,
    (5, 2): 0.517231671970585, (5, 3): 0.096059710526147, (5, 4): 0.386708617503269,
}
BETA = {
    (1, 0): 0.391752226571890,
    (2, 1): 0.368410593050371,
    (3, 2): 0.251891774271694,
    (4, 3): 0.544974750228521,
    (5, 3): 0.063692468666290, (5, 4): 0.226007483236906,
}
STAGES = 5


def positivity_floor(U, gamma, rho_min, p_min):
    """The floor above on an Euler state (B, dim + 2, ...)."""
    rho = torch.clamp(U[:, 0], min=rho_min)
    m = U[:, 1:-1]
    ke = 0.5 * (m * m).sum(dim=1) / rho
    E = torch.maximum(U[:, -1], p_min / (gamma - 1.0) + ke)
    return torch.cat([rho[:, None], m, E[:, None]], dim=1)


def ssprk54_step(op, U, dt, floor=None):
    """One step of the method from U = U^n; floor = (rho_min, p_min) applies
    the positivity floor to every stage U^(1..5)."""
    stages = [U]
    L = {}
    for i in range(1, STAGES + 1):
        acc = torch.zeros_like(U)
        for k in range(i):
            a, b = ALPHA.get((i, k), 0.0), BETA.get((i, k), 0.0)
            if a != 0.0:
                acc = acc + a * stages[k]
            if b != 0.0:
                if k not in L:
                    L[k] = op.rhs(stages[k])
                acc = acc + dt * b * L[k]
        if floor is not None:
            acc = positivity_floor(acc, op.phys.gamma, *floor)
        stages.append(acc)
    return stages[STAGES]

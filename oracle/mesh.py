"""Periodic Cartesian meshes, optionally with one 2:1-refined block (2-D).

The element map is the affine case of the paper's mapping x = X(xi) (Kernel
Architecture for Hyperbolic Terms): element e with lower corner x_e and widths
h_{e,l} has nodes x = x_e + (xi + 1) h / 2, Jacobian J_e = prod_l h_{e,l}/2 and
contravariant vectors Ja^l = (2 J_e / h_{e,l}) e_l, which satisfy the discrete
GCL trivially (constant per element).

Element order (shared convention with the HIP library, each side implements it
on its own): coarse cells are visited lexicographically (x fastest, then y,
then z); an unrefined cell emits one element, a refined cell emits its four
children in the order (0,0), (1,0), (0,1), (1,1) (x fastest).  Node order
inside an element is (k, j, i) with i fastest.

Faces:
* conforming faces normal to direction l are pairs (L, R) with L on the -xi_l
  side and R on the +xi_l side of the face;
* a 2:1 non-conforming face is a mortar record (coarse element, l, side of the
  coarse element the face sits on, the two fine elements ordered by increasing
  tangential coordinate).
"""

from dataclasses import dataclass, field

import numpy as np

from .refelem import gll


@dataclass
class Mesh:
    dim: int
    N: int
    lo: tuple
    hi: tuple
    nel: tuple
    corner: np.ndarray          # (E, dim)
    h: np.ndarray               # (E, dim)
    level: np.ndarray           # (E,)
    conf: list                  # per direction l: (L, R) int64 arrays
    mortars: list = field(default_factory=list)  # dicts, see module doc

    @property
    def E(self):
        return self.corner.shape[0]

    @property
    def n(self):
        return self.N + 1

    @property
    def Np(self):
        return self.n ** self.dim

    def jac(self):
        """J_e = prod_l h_{e,l} / 2, shape (E,)."""
        return np.prod(self.h / 2.0, axis=1)

    def coords(self):
        """Node coordinates, shape (dim, E, n, .., n) with axes (k, j, i)."""
        xi, _, _ = gll(self.N)
        n = self.n
        out = []
        for d in range(self.dim):
            # axis of direction d in the (k, j, i) node block
            ax = self.dim - 1 - d
            shape = [1] * self.dim
            shape[ax] = n
            x1 = xi.reshape(shape)
            x = self.corner[:, d].reshape((-1,) + (1,) * self.dim) + \
                (x1[None] + 1.0) * self.h[:, d].reshape((-1,) + (1,) * self.dim) / 2.0
            out.append(np.broadcast_to(x, (self.E,) + (n,) * self.dim).copy())
        return np.stack(out)

    def hmin(self):
        return float(np.min(self.h))


def cartesian_mesh(dim, N, nel, lo, hi, patch_lo=None, patch_hi=None):
    """Build the periodic box [lo, hi] with nel coarse cells per direction.

    patch_lo/patch_hi (2-D only) give a block of coarse cells [patch_lo,
    patch_hi) refined once into 2x2 children.
    """
    nel = tuple(int(v) for v in nel)
    lo = tuple(float(v) for v in lo)
    hi = tuple(float(v) for v in hi)
    h0 = np.array([(hi[d] - lo[d]) / nel[d] for d in range(dim)])
    refined = np.zeros(nel[::-1], dtype=bool)  # indexed [cz][cy][cx] / [cy][cx]
    if patch_lo is not None and tuple(patch_lo) != tuple(patch_hi):
        if dim != 2:
            raise ValueError("refined patch only in 2-D")
        refined[patch_lo[1]:patch_hi[1], patch_lo[0]:patch_hi[0]] = True

    corner, hs, level, key = [], [], [], {}
    cells = np.ndindex(*nel[::-1])
    for idx in cells:
        c = idx[::-1]  # (cx, cy[, cz]), x fastest in the traversal
        if dim == 2 and refined[c[1], c[0]]:
            for fy in range(2):
                for fx in range(2):
                    f = (2 * c[0] + fx, 2 * c[1] + fy)
                    key[(1,) + f] = len(corner)
                    corner.append([lo[d] + f[d] * h0[d] / 2 for d in range(dim)])
                    hs.append(list(h0 / 2))
                    level.append(1)
        else:
            key[(0,) + tuple(c)] = len(corner)
            corner.append([lo[d] + c[d] * h0[d] for d in range(dim)])
            hs.append(list(h0))
            level.append(0)
    corner = np.array(corner, dtype=np.float64)
    hs = np.array(hs, dtype=np.float64)
    level = np.array(level, dtype=np.int64)

    def is_refined(c):
        return dim == 2 and bool(refined[c[1], c[0]])

    conf = [([], []) for _ in range(dim)]
    mortars = []
    for (lev, *ic), e in key.items():
        for l in range(dim):
            if lev == 0:
                c = list(ic)
                c[l] = (c[l] + 1) % nel[l]
                if not is_refined(c):
                    conf[l][0].append(e)
                    conf[l][1].append(key[(0,) + tuple(c)])
                else:
                    t = 1 - l
                    fine = []
                    for s in range(2):
                        f = [0, 0]
                        f[l] = 2 * c[l]
                        f[t] = 2 * ic[t] + s
                        fine.append(key[(1,) + tuple(f)])
                    mortars.append(dict(coarse=e, l=l, side=1, fine=fine))
                # the coarse element's -l face against a refined cell
                c2 = list(ic)
                c2[l] = (c2[l] - 1) % nel[l]
                if is_refined(c2):
                    t = 1 - l
                    fine = []
                    for s in range(2):
                        f = [0, 0]
                        f[l] = 2 * c2[l] + 1
                        f[t] = 2 * ic[t] + s
                        fine.append(key[(1,) + tuple(f)])
                    mortars.append(dict(coarse=e, l=l, side=0, fine=fine))
            else:
                f = list(ic)
                f[l] = (f[l] + 1) % (2 * nel[l])
                parent = [v // 2 for v in f]
                if is_refined(parent):
                    conf[l][0].append(e)
                    conf[l][1].append(key[(1,) + tuple(f)])
                # fine/coarse faces are recorded from the coarse side above
    conf = [(np.array(L, dtype=np.int64), np.array(R, dtype=np.int64)) for (L, R) in conf]
    return Mesh(dim=dim, N=N, lo=lo, hi=hi, nel=nel, corner=corner, h=hs,
                level=level, conf=conf, mortars=mortars)

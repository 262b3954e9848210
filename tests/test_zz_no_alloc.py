"""dg_integrals_noalloc (fixed per-GPU scratch, no allocation in the call)
against dg_integrals on the same inputs: two calls in a row, the second on a
smaller input, and the limit of the fixed scratch."""

import numpy as np
import pytest
import torch

import dginputs as di
from paper_2605_26388_amd import Solver
from paper_2605_26388_amd._abi import DG_ERR_UNSUPPORTED, DGError

pytestmark = pytest.mark.gpu


def _case(dim, N, nel, batch, precision, seed):
    lo, hi = (0.0,) * dim, (2 * np.pi,) * dim
    s = Solver(dim, N, nel, lo, hi, batch=batch, precision=precision)
    X = s.node_coords().cpu().numpy()
    base = di.random_euler(X, lo, hi)
    U = np.stack([di.perturb_density(base, seed + b) for b in range(batch)])
    return s, torch.tensor(U).to(s.device, s.dtype).contiguous()


def test_noalloc_integrals_match_two_calls_second_smaller():
    big = _case(3, 3, (5, 4, 3), 3, "f64", 11)
    small = _case(2, 2, (3, 2), 1, "f32", 23)
    for s, U in (big, small):
        want = s.integrals(U)
        out = torch.full((s.batch, s.nv + 1), float("nan"), dtype=torch.float64, device=s.device)
        s.integrals_noalloc(U, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"noalloc integrals: dim {s.dim} N={s.N} batch {s.batch} {s.precision}: "
              f"max |diff| {np.abs(got - want).max():.3e}", flush=True)
        # same kernels, same partial layout, same summation order: identical bits
        assert np.array_equal(got, want), (got, want)
        assert np.isfinite(got).all()
    for s, _ in (big, small):
        s.close()


def test_noalloc_integrals_reject_batch_beyond_scratch():
    lo, hi = (0.0,) * 3, (1.0,) * 3
    s = Solver(3, 1, (2, 2, 2), lo, hi, batch=86)  # 86 * 6 rows > 512
    U = torch.ones(s.shape, dtype=s.dtype, device=s.device)
    out = torch.zeros((s.batch, s.nv + 1), dtype=torch.float64, device=s.device)
    with pytest.raises(DGError) as ei:
        s.integrals_noalloc(U, out)
    assert ei.value.code == DG_ERR_UNSUPPORTED
    assert "scratch" in str(ei.value)
    s.close()

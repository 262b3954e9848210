"""dg_create's synchronous argument checks (host logic, no GPU needed): every
invalid or unsupported descriptor is rejected with its error code and a
message before any device is touched; a valid descriptor passes the checks
(it then fails only on the device query when no GPU is present)."""

import ctypes
import os

import pytest

from paper_2605_26388_amd import _abi

pytestmark = pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="libdg.so not built")


def desc(dim=3, degree=3, nel=(4, 4, 4), physics=_abi.DG_EULER, precision=_abi.DG_F64, batch=1,
         patch=None, gamma=1.4, mu=0.0, prandtl=0.72, mech=None, volume=_abi.DG_VOLUME_STANDARD,
         rho_floor=0.0, p_floor=0.0, vib=None, warp=0.0, bc=None, bc_state=None):
    d = _abi.Desc()
    d.dim, d.degree, d.physics, d.precision, d.batch = dim, degree, physics, precision, batch
    for l in range(3):
        d.nel[l] = nel[l] if l < len(nel) else 1
        d.lo[l], d.hi[l] = 0.0, 1.0
    if patch:
        for l in range(2):
            d.patch_lo[l], d.patch_hi[l] = patch[0][l], patch[1][l]
    d.gamma, d.mu, d.prandtl = gamma, mu, prandtl
    if mech == "air5":
        import dginputs as di
        from paper_2605_26388_amd.solver import mechanism_struct
        d._mech_keep = mechanism_struct(di.preset_mechanism(di.PRESETS["air5_2d"]))
        mech = ctypes.pointer(d._mech_keep)
    d.mech = mech
    d.newton_max_iter, d.newton_tol, d.device = 25, 1e-13, 0
    d.volume = volume
    d.rho_floor, d.p_floor = rho_floor, p_floor
    d.warp = warp
    for q, v in enumerate(bc or ()):
        d.bc[q] = v
    for q, v in enumerate(bc_state or ()):
        d.bc_state[q] = v
    if vib == "air5":
        import dginputs as di
        from paper_2605_26388_amd.solver import vibration_struct
        d._vib_keep = vibration_struct(di.air5_vibration(di.preset_mechanism(di.PRESETS["air5_2t_2d"])))
        d.vib = ctypes.pointer(d._vib_keep)
    return d


def create(d):
    lib = _abi.load()
    ctx = ctypes.c_void_p()
    rc = lib.dg_create(ctypes.byref(d), ctypes.byref(ctx))
    if rc == _abi.DG_OK:  # a GPU is present: the descriptor was valid
        lib.dg_destroy(ctx)
    return rc, lib.dg_last_error().decode()


@pytest.mark.parametrize("kw,code,msg", [
    (dict(nel=(0, 4, 4)), _abi.DG_ERR_ARG, "nel"),                     # empty mesh
    (dict(batch=0), _abi.DG_ERR_ARG, "batch"),                          # empty batch
    (dict(degree=0), _abi.DG_ERR_UNSUPPORTED, "degree"),
    (dict(degree=8), _abi.DG_ERR_UNSUPPORTED, "degree"),
    (dict(dim=1, nel=(4,)), _abi.DG_ERR_UNSUPPORTED, "dim"),
    (dict(precision=7), _abi.DG_ERR_ARG, "precision"),
    (dict(gamma=1.0), _abi.DG_ERR_ARG, "gamma"),
    (dict(physics=9), _abi.DG_ERR_ARG, "physics"),
    (dict(physics=_abi.DG_NAVIER_STOKES, degree=5), _abi.DG_ERR_UNSUPPORTED, "Navier-Stokes"),
    (dict(physics=_abi.DG_NAVIER_STOKES, prandtl=0.0), _abi.DG_ERR_ARG, "prandtl"),
    (dict(physics=_abi.DG_REACTING_EULER), _abi.DG_ERR_UNSUPPORTED, "reacting"),
    (dict(dim=2, nel=(8, 8), patch=((2, 2), (9, 4))), _abi.DG_ERR_ARG, "patch"),
    (dict(dim=2, nel=(8, 8), patch=((0, 2), (8, 4))), _abi.DG_ERR_UNSUPPORTED, "period"),
    # just above the 32-bit state addressing limit: 119^3 elements x 64 nodes x 5 x 8 B > 4 GiB
    (dict(nel=(119, 119, 119)), _abi.DG_ERR_UNSUPPORTED, "4 GiB"),
    (dict(volume=2), _abi.DG_ERR_ARG, "volume"),
    (dict(volume=_abi.DG_VOLUME_SPLIT, physics=_abi.DG_REACTING_EULER, dim=2, nel=(8, 8), mech="air5"),
     _abi.DG_ERR_UNSUPPORTED, "split"),
    (dict(rho_floor=-1e-6), _abi.DG_ERR_ARG, "floor"),
    (dict(p_floor=float("nan")), _abi.DG_ERR_ARG, "floor"),
    (dict(p_floor=float("inf")), _abi.DG_ERR_ARG, "floor"),
    (dict(physics=_abi.DG_REACTING_EULER, dim=2, nel=(8, 8), rho_floor=1e-6, mech="air5"),
     _abi.DG_ERR_UNSUPPORTED, "floor"),
    (dict(physics=_abi.DG_REACTING_2T, dim=2, nel=(8, 8), mech="air5"), _abi.DG_ERR_ARG, "vib"),
    (dict(physics=_abi.DG_REACTING_2T, dim=3, mech="air5", vib="air5"), _abi.DG_ERR_UNSUPPORTED, "2-D"),
    (dict(warp=0.3), _abi.DG_ERR_ARG, "warp"),
    (dict(warp=float("nan")), _abi.DG_ERR_ARG, "warp"),
    (dict(bc=(1, 0, 0, 0, 0, 0)), _abi.DG_ERR_ARG, "periodic"),
    (dict(bc=(7, 7, 0, 0, 0, 0)), _abi.DG_ERR_ARG, "dg_bc"),
    (dict(warp=0.05, physics=_abi.DG_NAVIER_STOKES, bc=(2, 2, 0, 0, 0, 0)), _abi.DG_ERR_UNSUPPORTED, "periodic"),
    (dict(warp=0.05, physics=_abi.DG_REACTING_EULER, dim=2, nel=(8, 8), mech="air5"), _abi.DG_ERR_UNSUPPORTED,
     "Euler or Navier-Stokes"),
    (dict(dim=2, nel=(8, 8), patch=((2, 2), (4, 4)), bc=(1, 1, 0, 0)), _abi.DG_ERR_UNSUPPORTED, "patch"),
    (dict(bc=(2, 3, 0, 0, 0, 0), bc_state=(1.0, 0.0, 0.0, 0.0, -1.0)), _abi.DG_ERR_ARG, "bc_state"),
])
def test_invalid_descriptors_rejected(kw, code, msg):
    rc, err = create(desc(**kw))
    assert rc == code, (rc, err)
    assert msg in err


def test_size_limit_boundary_and_precision():
    # 118^3 FP64 (4.2e9 B) is the largest cube that fits; 149^3 fits only in FP32
    for kw in (dict(nel=(118, 118, 118)), dict(nel=(149, 149, 149), precision=_abi.DG_F32)):
        rc, err = create(desc(**kw))
        assert rc in (_abi.DG_OK, _abi.DG_ERR_HIP, _abi.DG_ERR_OOM), (kw, rc, err)
    rc, err = create(desc(nel=(149, 149, 149)))
    assert rc == _abi.DG_ERR_UNSUPPORTED and "4 GiB" in err


def test_null_arguments():
    lib = _abi.load()
    d = desc()
    assert lib.dg_create(ctypes.byref(d), None) == _abi.DG_ERR_ARG
    assert lib.dg_create(None, None) == _abi.DG_ERR_ARG


@pytest.mark.parametrize("kw", [dict(), dict(volume=_abi.DG_VOLUME_SPLIT),
                                dict(dim=2, nel=(8, 8), patch=((2, 2), (4, 4)), volume=_abi.DG_VOLUME_SPLIT,
                                     precision=_abi.DG_F32),
                                dict(rho_floor=1e-6, p_floor=5e-7),
                                dict(physics=_abi.DG_REACTING_2T, dim=2, nel=(8, 8), mech="air5", vib="air5"),
                                dict(warp=0.05, bc=(1, 1, 2, 3, 0, 0), bc_state=(1.0, 0.0, 2.0, 0.0, 5.0)),
                                dict(warp=0.05, volume=_abi.DG_VOLUME_SPLIT),
                                dict(warp=0.05, precision=_abi.DG_F32),
                                dict(warp=0.05, physics=_abi.DG_NAVIER_STOKES, mu=0.01),
                                dict(warp=0.05, physics=_abi.DG_NAVIER_STOKES, mu=0.01, volume=_abi.DG_VOLUME_SPLIT)])
def test_valid_descriptor_passes_the_checks(kw):
    rc, err = create(desc(**kw))
    # no device here: the only failure left is the device query itself
    assert rc in (_abi.DG_OK, _abi.DG_ERR_HIP), (rc, err)

"""Host-side checks of the C ABI library (no GPU): it loads, exports every
function include/cfd.h declares, and the binding covers all of them."""
import ctypes
import os
import re

import pytest

from paper_2203_13760_amd import cfd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cfd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared()
    for required in ("cfd_state_init", "cfd_rhs", "cfd_rk3_step", "cfd_advance", "cfd_rhs_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(cfd.LIB_PATH):
        pytest.skip("libcfd.so not built")
    lib = ctypes.CDLL(cfd.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(cfd.EXPORTS)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(cfd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cfd, "_lib", None)
    with pytest.raises(RuntimeError):
        cfd.load()


# ---------------------------------------------------------------- host-side validation
# Every check below fails in the library's argument validation, before any HIP
# call, so it runs without a GPU.

def _lib_or_skip():
    if not os.path.exists(cfd.LIB_PATH):
        pytest.skip("libcfd.so not built")
    return cfd.load()


def _case(**kw):
    case = {"n": (32, 24, 16), "lo": (0.0, 0.0, 0.0), "hi": (1.0, 1.0, 1.0), "nh": 3, "gamma": 1.4,
            "mu": 1e-3, "prandtl": 0.72, "cfl": 0.5, "bc": (0,) * 6, "flags": 7}
    case.update(kw)
    return case


BAD_CONFIGS = [
    ("nh", dict(nh=2), "nh"),
    ("short axis", dict(n=(32, 2, 16)), "n >= nh"),
    ("zero cells", dict(n=(32, 0, 16)), "n must be"),
    ("empty box", dict(hi=(1.0, 0.0, 1.0)), "lo < hi"),
    ("boundary type", dict(bc=(0, 0, 3, 3, 0, 0)), "boundary"),
    ("unpaired periodic", dict(bc=(0, 1, 0, 0, 0, 0)), "pairs"),
    ("no active axis", dict(n=(1, 1, 1)), "no active axis"),
    ("gamma", dict(gamma=1.0), "gamma"),
    ("negative viscosity", dict(mu=-1.0), "mu"),
    ("prandtl", dict(prandtl=0.0), "prandtl"),
    ("cfl zero", dict(cfl=0.0), "cfl"),
    ("cfl above one", dict(cfl=1.5), "cfl"),
    ("unknown flag", dict(flags=1024), "flag"),
    ("safe reconstruction with roe", dict(flags=1 | 16 | 512), "SAFE_RECON"),
    ("rusanov-nn without weno3", dict(flags=1 | 256), "Rusanov-NN"),
    ("rusanov-nn with rusanov", dict(flags=1 | 32 | 64 | 256), "Rusanov-NN"),
    ("rusanov-nn with roe", dict(flags=1 | 16 | 32 | 256), "Rusanov-NN"),
    ("roe with wenoz", dict(flags=1 | 8 | 16), "WENO5-JS"),
    ("roe with rusanov", dict(flags=1 | 16 | 64), "WENO5-JS"),
    ("wenoz with weno3", dict(flags=1 | 8 | 32), "WENO5-Z"),
    ("too many faces", dict(n=(2048, 2048, 600)), "too large"),
]


@pytest.mark.parametrize("label,kw,msg", BAD_CONFIGS, ids=[b[0] for b in BAD_CONFIGS])
def test_create_rejects_bad_config(label, kw, msg):
    _lib_or_skip()
    with pytest.raises(cfd.CfdError) as e:
        cfd.cfd_create(_case(**kw))
    assert e.value.code == cfd.CFD_EINVAL
    assert msg in cfd.cfd_last_error()


@pytest.mark.parametrize("label,kw,msg", BAD_CONFIGS[:4], ids=[b[0] for b in BAD_CONFIGS[:4]])
def test_footprint_rejects_bad_config(label, kw, msg):
    _lib_or_skip()
    with pytest.raises(cfd.CfdError):
        cfd.cfd_batch_footprint(_case(**kw))


@pytest.mark.parametrize("n", [(32, 24, 16), (64, 48, 1), (200, 1, 1)])
def test_footprint_counts_the_grid_buffers(n):
    """U, U1, U2, R (5 components each; a second accumulator R2 on grids with
    three active axes) and the three stage primitives (6 each) on the padded
    grid, the CFL slots and the control block, each rounded up to the arena
    alignment."""
    _lib_or_skip()
    need = cfd.cfd_batch_footprint(_case(n=n))
    padded = 1
    for d in range(3):
        padded *= n[d] + 6 if n[d] > 1 else 1
    base = 8 * padded * (43 if min(n) > 1 else 38)
    assert base <= need <= base + 8 * 256 + 16 + 16 * 256, (need, base)


def test_entry_points_reject_null_arguments():
    lib = _lib_or_skip()
    null = ctypes.c_void_p(0)
    for name, args in [("cfd_rhs", (null, null, null, null)),
                       ("cfd_rk3_step", (null, null, ctypes.c_double(0.0), null, null)),
                       ("cfd_advance", (null, null, ctypes.c_int32(1), ctypes.c_double(0.0), null, null)),
                       ("cfd_rhs_adjoint", (null, null, null, null, null)),
                       ("cfd_rk3_step_stages", (null, null, ctypes.c_double(1e-3), null, null, null)),
                       ("cfd_rk3_step_adjoint_stages", (null, null, null, null, ctypes.c_double(1e-3), null, null,
                                                        null)),
                       ("cfd_rk3_step_prims", (null, null, ctypes.c_double(1e-3), null, null)),
                       ("cfd_rk3_step_adjoint_prims", (null, null, ctypes.c_double(1e-3), null, null, null)),
                       ("cfd_set_nn_weights", (null, null, null)),
                       ("cfd_state_init", (null, null, null, null))]:
        assert getattr(lib, name)(*args) == cfd.CFD_EINVAL, name
        assert cfd.cfd_last_error() != ""


def test_noalloc_step_rejects_before_device_work():
    """The allocation-free step validates its configuration, and the grid
    against its static scratch, before any HIP call."""
    _lib_or_skip()
    fake = ctypes.c_void_p(8)  # never dereferenced: every case fails validation first
    lib = cfd.load()
    for kw, msg in [(dict(nh=2), "nh"), (dict(n=(78, 78, 78)), "too large"), (dict(flags=1 | 32 | 256), "Rusanov-NN")]:
        cfg = cfd.make_config(_case(**kw))
        rc = lib.cfd_rk3_step_noalloc(ctypes.byref(cfg), fake, ctypes.c_double(0.0), ctypes.c_void_p(0),
                                      ctypes.c_void_p(0))
        assert rc in (cfd.CFD_EINVAL, cfd.CFD_EUNSUPPORTED), kw
        assert msg in cfd.cfd_last_error(), (kw, cfd.cfd_last_error())
    assert lib.cfd_rk3_step_noalloc(ctypes.byref(cfd.make_config(_case())), ctypes.c_void_p(0), ctypes.c_double(0.0),
                                    ctypes.c_void_p(0), ctypes.c_void_p(0)) == cfd.CFD_EINVAL
    assert cfd.CFD_NOALLOC_MAX_PADDED_CELLS == 386309

"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/cgp.h, and sizes/validates configurations without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgp.h")
LIB = os.path.join(ROOT, "paper_1308_3290_amd", "libcgp.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcgp.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:cgp_status|const char\*)\s+(cgp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cgp_create", "cgp_step", "cgp_adjoint_step", "cgp_workspace_size",
                     "cgp_ensemble_step", "cgp_diagnostics", "cgp_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1308_3290_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        if name in _lib.OPTIONAL_SIGNATURES:
            continue
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"
    assert "gfx950" in lib.cgp_version().decode()


def test_measurement_build_exports_the_same_boundary_and_the_stamps():
    """libcgp_stamps.so exports every declared function, cgp_phase_stamps
    included; libcgp.so does not have cgp_phase_stamps."""
    from paper_1308_3290_amd import _lib
    if not os.path.exists(_lib.STAMPS_LIB_PATH):
        pytest.skip("libcgp_stamps.so not built")
    stamps = ctypes.CDLL(_lib.STAMPS_LIB_PATH)
    names = declared_functions()
    assert "cgp_phase_stamps" in names
    for name in names:
        assert hasattr(stamps, name), name
        assert name in _lib.SIGNATURES or name in _lib.OPTIONAL_SIGNATURES, name
    assert not hasattr(ctypes.CDLL(LIB), "cgp_phase_stamps")


def _cfg(**kw):
    from paper_1308_3290_amd.api import make_config
    base = dict(nx=64, ny=128, level=1, nlayers=1, dtype="f64", inv_re=1 / 450, inv_ro=1 / 0.0036,
                dt=1e-4)
    base.update(kw)
    return make_config(**base)


def test_workspace_size_is_positive_and_grows():
    from paper_1308_3290_amd.api import cgp_workspace_size
    a = cgp_workspace_size(_cfg())
    b = cgp_workspace_size(_cfg(nx=128, ny=256))
    c = cgp_workspace_size(_cfg(nlayers=2, f1=2000, f2=500))
    assert 0 < a < b and c > a
    assert a % 256 == 0


def test_workspace_shrinks_with_the_coarsening_level():
    """512 x 1024 at levels 0-3 (c = 1 .. 8, all fused-kernel sizes): the fine
    stage buffers stay, the coarse spectra and transform tables shrink."""
    from paper_1308_3290_amd.api import cgp_workspace_size
    sizes = [cgp_workspace_size(_cfg(nx=512, ny=1024, level=lv)) for lv in range(4)]
    assert all(a > b > 0 for a, b in zip(sizes, sizes[1:]))


@pytest.mark.parametrize("kw,status", [
    (dict(nx=65), 1),                  # not divisible by 2^level
    (dict(nlayers=3), 1),
    (dict(dtype=7), 1),
    (dict(level=-1), 1),
    (dict(nx=80, ny=160, level=0), 2),  # 80 = 5 * 16: radix 5 unsupported
    (dict(nx=8, ny=16, level=2), 2),    # coarse 2 x 4
    (dict(nx=4096, ny=4096, level=0), 2),
    (dict(inv_re=float("nan")), 1),
    (dict(inv_re=-1.0), 1),
    (dict(cfl=-0.5), 1),
    (dict(cfl=float("inf")), 1),
])
def test_invalid_configs_return_status(kw, status):
    from paper_1308_3290_amd.api import CGPError, cgp_workspace_size
    with pytest.raises(CGPError) as e:
        cgp_workspace_size(_cfg(**kw))
    assert e.value.status == status
    assert str(e.value)


def test_reserved_field_and_null_pointers():
    from paper_1308_3290_amd import _lib
    lib = _lib.load()
    cfg = _cfg()
    cfg.reserved = 1
    n = ctypes.c_size_t()
    assert lib.cgp_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == _lib.CGP_ERR_INVALID
    cfg.reserved = 0
    assert lib.cgp_workspace_size(ctypes.byref(cfg), None) == _lib.CGP_ERR_INVALID
    assert lib.cgp_step(None, None, None, None, 1, None) == _lib.CGP_ERR_INVALID
    assert lib.cgp_destroy(None) == _lib.CGP_OK
    h = ctypes.c_void_p()
    # NULL workspace is rejected before any device call
    assert lib.cgp_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == _lib.CGP_ERR_INVALID


def test_ensemble_offsets_pack_members_in_order():
    from paper_1308_3290_amd.api import cgp_ensemble_offsets, cgp_ensemble_workspace_size
    cfgs = [_cfg(nx=64, ny=128), _cfg(nx=96, ny=192), _cfg(nx=128, ny=256)]
    offs, tot = cgp_ensemble_offsets(cfgs)
    sizes = [65 * 129, 97 * 193, 129 * 257]
    assert offs == [0, sizes[0], sizes[0] + sizes[1]] and tot == sum(sizes)
    assert cgp_ensemble_workspace_size(cfgs) > 0
    from paper_1308_3290_amd.api import CGPError
    with pytest.raises(CGPError):
        cgp_ensemble_offsets([_cfg(), _cfg(dtype="f32")])


def test_tape_size():
    from paper_1308_3290_amd.api import cgp_tape_size
    assert cgp_tape_size(_cfg(), 20) == (6 * 20 + 4) * 65 * 129 * 8


def test_adaptive_step_config_and_fixed_step_adjoint():
    # an adaptive (cfl > 0) configuration is valid for the forward step and
    # gets a step-state region; the adjoint differentiates fixed steps only
    from paper_1308_3290_amd.api import CGPError, cgp_tape_size, cgp_workspace_size
    assert cgp_workspace_size(_cfg(cfl=0.5)) == cgp_workspace_size(_cfg())
    assert cgp_tape_size(_cfg(), 20) > 0
    with pytest.raises(CGPError) as e:
        cgp_tape_size(_cfg(cfl=0.5), 20)
    assert e.value.status == 2
    from paper_1308_3290_amd import _lib
    lib = _lib.load()
    out = ctypes.c_void_p()
    assert lib.cgp_time_state(None, out, None) == _lib.CGP_ERR_INVALID


@pytest.mark.parametrize("kw,status", [
    (dict(solver=2), 1),
    (dict(solver=1, mg_cycles=-1), 1),
    (dict(solver=1, mg_cycles=5000), 1),
    (dict(solver=1, nlayers=2, f1=2000, f2=500), 2),   # multigrid: one layer only
])
def test_multigrid_config_validation(kw, status):
    from paper_1308_3290_amd.api import CGPError, cgp_workspace_size
    with pytest.raises(CGPError) as e:
        cgp_workspace_size(_cfg(**kw))
    assert e.value.status == status


def test_multigrid_workspace_and_limits():
    from paper_1308_3290_amd.api import (CGPError, cgp_ensemble_workspace_size, cgp_tape_size,
                                         cgp_workspace_size)
    assert cgp_workspace_size(_cfg(solver=1)) > cgp_workspace_size(_cfg())
    with pytest.raises(CGPError) as e:
        cgp_tape_size(_cfg(solver=1), 10)
    assert e.value.status == 2
    with pytest.raises(CGPError) as e:  # single basin only
        cgp_ensemble_workspace_size([_cfg(solver=1), _cfg(solver=1)])
    assert e.value.status == 2
    with pytest.raises(CGPError):       # members share the solver
        cgp_ensemble_workspace_size([_cfg(solver=1), _cfg()])


def test_fused_rows_validation_and_workspace():
    """cgp_config.fused_rows: 0, 2 or 4, shared by every member; 4 rows per
    fused block at c = 2 changes the fused blocks (fewer step-state slots),
    not the spectra, so the workspace is no larger."""
    from paper_1308_3290_amd.api import (CGPError, cgp_ensemble_workspace_size,
                                         cgp_workspace_size)
    for bad in (1, 3, 8, -2):
        with pytest.raises(CGPError) as e:
            cgp_workspace_size(_cfg(level=1, fused_rows=bad))
        assert e.value.status == 1
    with pytest.raises(CGPError):
        cgp_ensemble_workspace_size([_cfg(level=1, fused_rows=4), _cfg(level=1)])
    two = cgp_workspace_size(_cfg(level=1))
    assert cgp_workspace_size(_cfg(level=1, fused_rows=2)) == two
    assert cgp_workspace_size(_cfg(level=1, fused_rows=4)) <= two


def test_noalloc_step_rejects_an_oversized_workspace_on_the_host():
    """cgp_step_noalloc checks the workspace size against its static scratch
    before any device work (no GPU needed for the refusal)."""
    import torch
    from paper_1308_3290_amd._lib import CGP_ERR_INVALID, CGPError
    from paper_1308_3290_amd.api import cgp_step_noalloc, make_config
    cfg = make_config(1024, 1024, level=0, nlayers=2, f1=10.0, f2=5.0, inv_re=1e-3, dt=1e-5)
    host = torch.zeros(4)  # never dereferenced: the call fails before touching memory
    with pytest.raises(CGPError) as ei:
        cgp_step_noalloc(cfg, host, host, None, 1, stream=_NoStream())
    assert ei.value.status == CGP_ERR_INVALID and "static scratch" in str(ei.value)


class _NoStream:
    cuda_stream = 0

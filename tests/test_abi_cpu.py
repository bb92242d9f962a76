"""The C ABI without a GPU: the library loads, exports every declared symbol,
and its host-only validation and sizing behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2503_13961_amd import native as N
from paper_2503_13961_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "bgt.h")).read()
    return sorted(set(re.findall(r"\b(bgt_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(N.EXPORTS) == names


def test_binding_constants_match_the_header():
    """The binding's copies of the header's sizes (a state-layout array one
    entry short would be overrun by bgt_state_layout)."""
    import re
    hdr = open(os.path.join(ROOT, "include", "bgt.h")).read()
    for name in ("BGT_STATE_FIELDS", "BGT_MAX_VIEWS", "BGT_MAX_ADAM_GROUPS", "BGT_FLAG_NO_BOUNDARY", "BGT_NUM_STAGES"):
        m = re.search(rf"#define {name} (\d+)", hdr)
        assert m and int(m.group(1)) == getattr(N, name), name


def test_default_config_is_valid_and_checks_reject_bad_values():
    c = N.bgt_default_config()
    assert N.bgt_validate_config(c) == N.BGT_OK
    assert (c.tess_level, c.tile, c.z_near) == (4, 16, np.float32(0.2))
    for field, bad in (("tile", 12), ("tess_level", 0), ("tess_level", 9), ("batch", 48),
                       ("alpha_max", 1.0), ("g_min", 0.0), ("z_near", 0.0), ("pair_factor", 0.0)):
        assert N.bgt_validate_config(N.bgt_default_config(**{field: bad})) == N.BGT_E_INVALID, field
    assert N.bgt_validate_config(N.bgt_default_config(bg=(0, float("nan"), 0))) == N.BGT_E_INVALID
    for tile, batch in ((8, 32), (8, 64), (16, 128), (32, 128)):
        assert N.bgt_validate_config(N.bgt_default_config(tile=tile, batch=batch)) == N.BGT_OK
    # one loader thread per batch slot: an 8-px tile has 64
    assert N.bgt_validate_config(N.bgt_default_config(tile=8, batch=128)) == N.BGT_E_INVALID
    # flags: only the no-boundary bit is defined
    assert N.bgt_validate_config(N.bgt_default_config(flags=N.BGT_FLAG_NO_BOUNDARY)) == N.BGT_OK
    assert N.bgt_validate_config(N.bgt_default_config(flags=2)) == N.BGT_E_INVALID
    # a misspelt or unknown option is an error, not a silently ignored attribute
    with pytest.raises(TypeError):
        N.bgt_default_config(no_boundary=True)


def test_prims_and_views_validation():
    c = N.bgt_default_config()
    good = N.make_prims(2, 10, 1, 1, 1, 1, 1, 1)
    assert N.bgt_validate_prims(good, c) == N.BGT_OK
    assert N.bgt_validate_prims(N.make_prims(0, 10, 1, 1, 1, 1, 1, 1), c) == N.BGT_E_INVALID
    assert N.bgt_validate_prims(N.make_prims(6, 10, 1, 1, 1, 1, 1, 1), c) == N.BGT_E_INVALID
    assert N.bgt_validate_prims(N.make_prims(2, 0, 1, 1, 1, 1, 1, 1), c) == N.BGT_E_INVALID
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 0, 1, 1), c) == N.BGT_E_INVALID
    # attribute maps of resolution 1 or 3; SH colour of degree 0..3 with its array
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, attr_res=3), c) == N.BGT_OK
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, attr_res=2), c) == N.BGT_E_UNSUPPORTED
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, sh_degree=3, sh=1), c) == N.BGT_OK
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, sh_degree=3), c) == N.BGT_E_INVALID
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, sh_degree=4, sh=1), c) == N.BGT_E_UNSUPPORTED
    assert N.bgt_validate_prims(N.make_prims(2, 10, 1, 1, 1, 1, 1, 1, sh_degree=-1, sh=1), c) == N.BGT_E_INVALID
    # sub-triangle ids must fit 24 bits
    assert N.bgt_validate_prims(N.make_prims(2, 1 << 20, 1, 1, 1, 1, 1, 1), c) == N.BGT_E_INVALID
    wh = np.array([[800, 800], [37, 1]], np.int32)
    assert N.bgt_validate_views(N.make_views(wh, 1)) == N.BGT_OK
    assert N.bgt_validate_views(N.make_views(wh, 0)) == N.BGT_E_INVALID
    for bad in ([[0, 5]], [[20000, 2]], [[4096, 4096]]):
        assert N.bgt_validate_views(N.make_views(np.array(bad, np.int32), 1)) == N.BGT_E_INVALID
    many = np.ones((N.BGT_MAX_VIEWS + 1, 2), np.int32)
    assert N.bgt_validate_views(N.make_views(many, 1)) == N.BGT_E_INVALID


def test_host_only_context_sizes_state_and_refuses_work():
    ctx = N.bgt_create(N.bgt_default_config(), -1)
    try:
        sc, cams, _ = S.workload("sphere2k_16v_800")
        pr = N.make_prims(2, sc.num_prims, 1, 1, 1, 1, 1, 1)
        vw = N.make_views(cams.wh, 1)
        n = N.bgt_state_size(ctx, pr, vw)
        lay = N.bgt_state_layout(ctx, pr, vw)
        assert lay["end"] == n
        offs = [lay[k] for k in N.STATE_FIELD_NAMES]
        assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
        npx = cams.num_pixels
        assert lay["I_tri"] - lay["zbuf"] >= 8 * npx and lay["rec"] + 64 * npx <= lay["gkey"]
        with pytest.raises(N.BgtError) as e:
            N.bgt_render_fwd(ctx, pr, vw, 1, 1, n, 0)
        assert e.value.status == N.BGT_E_INVALID
        assert "host-only" in N.bgt_last_error(ctx)
    finally:
        N.bgt_destroy(ctx)


def test_lattice_option_validation_and_state_size():
    """The lattice variant: m in 2..16 (0 = pixel Gaussians); the record
    arrays grow by V P NL, NL = (M+1)(M+2)/2, M = L (m - 1); a view whose
    pixels plus lattice Gaussians exceed 24-bit ids is refused."""
    assert N.bgt_default_config().lattice == 0
    for m, want in ((0, N.BGT_OK), (2, N.BGT_OK), (16, N.BGT_OK), (1, N.BGT_E_INVALID), (17, N.BGT_E_INVALID),
                    (-2, N.BGT_E_INVALID)):
        assert N.bgt_validate_config(N.bgt_default_config(lattice=m)) == want, m
    sc, cams, _ = S.workload("sphere2k_16v_800")
    pr = N.make_prims(2, sc.num_prims, 1, 1, 1, 1, 1, 1)
    vw = N.make_views(cams.wh, 1)
    lays = {}
    for m in (0, 4):
        ctx = N.bgt_create(N.bgt_default_config(lattice=m), -1)
        try:
            lays[m] = N.bgt_state_layout(ctx, pr, vw)
        finally:
            N.bgt_destroy(ctx)
    NR = cams.num_pixels + cams.n_views * sc.num_prims * 91
    assert lays[4]["gkey"] - lays[4]["rec"] >= 64 * NR and lays[4]["T_final"] - lays[4]["gkey"] >= 8 * NR
    assert lays[4]["end"] > lays[0]["end"]
    ctx = N.bgt_create(N.bgt_default_config(lattice=16), -1)
    try:
        big = N.make_views(np.array([[4000, 4000]], np.int32), 1)
        with pytest.raises(N.BgtError) as e:
            N.bgt_state_size(ctx, N.make_prims(2, 3000, 1, 1, 1, 1, 1, 1), big)
        assert e.value.status == N.BGT_E_INVALID and "2^24" in N.bgt_last_error(ctx)
    finally:
        N.bgt_destroy(ctx)


def test_create_rejects_bad_device_and_config():
    with pytest.raises(N.BgtError):
        N.bgt_create(N.bgt_default_config(tile=7), -1)
    h = C.c_void_p()
    assert N.lib().bgt_create(None, -1, C.byref(h)) == N.BGT_OK
    N.bgt_destroy(h)


def test_training_step_entry_points_validate_on_the_host():
    """bgt_loss sizes its workspace (three float maps per pixel-channel and
    two doubles per 32x16 tile) and both training entry points reject bad
    arguments, and any work on a host-only context, before enqueuing."""
    wh = np.array([[800, 800], [37, 29]], np.int32)
    vw = N.make_views(wh, None)
    px = 800 * 800 + 37 * 29
    tiles = 25 * 50 + 2 * 2

    def a256(x):
        return (x + 255) // 256 * 256
    assert N.bgt_loss_workspace_size(vw) == a256(9 * 4 * px) + a256(16 * tiles)
    with pytest.raises(N.BgtError):
        N.bgt_loss_workspace_size(N.make_views(np.array([[0, 5]], np.int32), None))
    ctx = N.bgt_create(N.bgt_default_config(), -1)
    try:
        ws = N.bgt_loss_workspace_size(vw)
        for lam, nbytes, status in ((1.5, ws, N.BGT_E_INVALID), (0.2, ws - 1, N.BGT_E_NOMEM),
                                    (0.2, ws, N.BGT_E_INVALID)):
            with pytest.raises(N.BgtError) as e:
                N.bgt_loss(ctx, vw, 1, 1, lam, 1, 1, 1, nbytes, 0)
            assert e.value.status == status
        assert "host-only" in N.bgt_last_error(ctx)
        g = N.bgt_adam_group(1, 1, 1, 1, 10, 1e-3, 0)
        for groups, b1, b2, eps in (([g], 1.0, 0.999, 1e-15), ([g], 0.9, -0.1, 1e-15), ([g], 0.9, 0.999, -1.0),
                                    ([g] * 9, 0.9, 0.999, 1e-15),
                                    ([N.bgt_adam_group(None, 1, 1, 1, 10, 1e-3, 0)], 0.9, 0.999, 1e-15),
                                    ([g], 0.9, 0.999, 1e-15)):
            with pytest.raises(N.BgtError) as e:
                N.bgt_adam_step(ctx, groups, b1, b2, eps, 1, 0)
            assert e.value.status == N.BGT_E_INVALID
        assert "host-only" in N.bgt_last_error(ctx)
    finally:
        N.bgt_destroy(ctx)


def test_bench_measures_one_gpu_only():
    """bench.py --gpus N with N > 1 exits with a message instead of timing."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout

"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/*.h, and rejects invalid arguments with the
documented status before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gs.h", "gs_nn.h")]
LIB = os.path.join(ROOT, "paper_2409_09295_amd", "libgsmi.so")


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def gs():
    if not os.path.exists(LIB):
        pytest.fail("libgsmi.so is not built (run python -m paper_2409_09295_amd.build)")
    from paper_2409_09295_amd import gs as _gs
    return _gs


def test_every_declared_symbol_is_exported(gs):
    names = _declared()
    assert len(names) >= 30
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    # and the Python binding wraps every one of them
    assert set(names) <= set(gs.EXPORTED), set(names) - set(gs.EXPORTED)


def test_status_strings(gs):
    lib = gs.lib()
    assert lib.gs_status_string(0) == b"GS_OK"
    assert lib.gs_status_string(2) == b"GS_ERR_CAPACITY"
    assert lib.gs_status_string(99) == b"GS_ERR_UNKNOWN"
    assert b"gfx950" in lib.gs_version()


def _views(gs, sizes, tile=16):
    arr = (gs.gs_camera * len(sizes))()
    for i, (w, h) in enumerate(sizes):
        arr[i].fx = arr[i].fy = 100.0
        arr[i].cx, arr[i].cy = w / 2, h / 2
        arr[i].width, arr[i].height = w, h
        arr[i].R[0] = arr[i].R[4] = arr[i].R[8] = 1.0
    v = gs.gs_views(ctypes.cast(arr, ctypes.c_void_p), 0xDEAD0000, len(sizes), tile)
    v._keep = arr
    return v


def test_tile_and_pixel_counts(gs):
    lib = gs.lib()
    v = _views(gs, [(160, 120), (100, 70), (1200, 680)])
    assert lib.gs_num_tiles(ctypes.byref(v)) == 10 * 8 + 7 * 5 + 75 * 43
    assert lib.gs_num_pixels(ctypes.byref(v)) == 160 * 120 + 100 * 70 + 1200 * 680
    bad = _views(gs, [(0, 10)])
    assert lib.gs_num_tiles(ctypes.byref(bad)) == -1


def test_workspace_sizes_grow(gs):
    lib = gs.lib()
    v = _views(gs, [(640, 480)])
    a = lib.gs_bin_sort_workspace_size(1000, ctypes.byref(v), 10000)
    b = lib.gs_bin_sort_workspace_size(50000, ctypes.byref(v), 10000)
    c = lib.gs_bin_sort_workspace_size(1000, ctypes.byref(v), 20000)
    assert 0 < a < b and a < c
    assert lib.gs_render_bwd_workspace_size(1000, ctypes.byref(v)) >= 36 * 1000
    assert lib.gs_bin_sort_workspace_size(-1, ctypes.byref(v), 10) == 0


FAKE = 0x7F0000000000   # never dereferenced: validation fails first


def _gauss(gs, n=10, deg=0):
    return gs.gs_gaussians(FAKE, FAKE, FAKE, FAKE, FAKE, n, deg)


def test_preprocess_argument_errors(gs):
    lib = gs.lib()
    v = _views(gs, [(64, 48)])
    proj = gs.gs_projected(FAKE, FAKE, FAKE, FAKE)
    assert lib.gs_preprocess(None, ctypes.byref(v), ctypes.byref(proj), None) == gs.GS_ERR_INVALID_ARGUMENT
    g = _gauss(gs, deg=4)
    assert lib.gs_preprocess(ctypes.byref(g), ctypes.byref(v), ctypes.byref(proj), None) == 1
    assert b"sh_degree" in lib.gs_last_error()
    g = _gauss(gs, n=-1)
    assert lib.gs_preprocess(ctypes.byref(g), ctypes.byref(v), ctypes.byref(proj), None) == 1
    g = _gauss(gs)
    g.means = None
    assert lib.gs_preprocess(ctypes.byref(g), ctypes.byref(v), ctypes.byref(proj), None) == 1
    v8 = _views(gs, [(64, 48)], tile=8)
    assert lib.gs_preprocess(ctypes.byref(_gauss(gs)), ctypes.byref(v8), ctypes.byref(proj),
                             None) == gs.GS_ERR_UNSUPPORTED
    v0 = _views(gs, [(64, 48)])
    v0.n_views = 0
    assert lib.gs_preprocess(ctypes.byref(_gauss(gs)), ctypes.byref(v0), ctypes.byref(proj), None) == 1
    vbig = _views(gs, [(64, 48)] * 65)
    assert lib.gs_preprocess(ctypes.byref(_gauss(gs)), ctypes.byref(vbig), ctypes.byref(proj), None) == 1
    # n * views must fit the 32-bit splat index
    g = _gauss(gs, n=1 << 31)
    v3 = _views(gs, [(64, 48)] * 3)
    assert lib.gs_preprocess(ctypes.byref(g), ctypes.byref(v3), ctypes.byref(proj), None) == 1


def test_bin_sort_argument_errors(gs):
    lib = gs.lib()
    v = _views(gs, [(64, 48)])
    proj = gs.gs_projected(FAKE, FAKE, FAKE, FAKE)
    bins = gs.gs_bins(FAKE, FAKE, FAKE, FAKE, 100)
    need = lib.gs_bin_sort_workspace_size(10, ctypes.byref(v), 100)
    # workspace too small -> capacity error naming the size
    st = lib.gs_bin_sort(ctypes.byref(proj), 10, ctypes.byref(v), ctypes.byref(bins), None, FAKE,
                         need - 1, None)
    assert st == gs.GS_ERR_CAPACITY
    assert str(need).encode() in lib.gs_last_error()
    # misaligned workspace
    st = lib.gs_bin_sort(ctypes.byref(proj), 10, ctypes.byref(v), ctypes.byref(bins), None, FAKE + 4,
                         need, None)
    assert st == 1
    bins.capacity = -5
    st = lib.gs_bin_sort(ctypes.byref(proj), 10, ctypes.byref(v), ctypes.byref(bins), None, FAKE,
                         need, None)
    assert st == 1
    # keys are optional; values, ranges and the device count are not
    bins = gs.gs_bins(FAKE, None, FAKE, FAKE, 100)
    st = lib.gs_bin_sort(ctypes.byref(proj), 10, ctypes.byref(v), ctypes.byref(bins), None, FAKE,
                         need, None)
    assert st == 1


def test_render_argument_errors(gs):
    lib = gs.lib()
    v = _views(gs, [(64, 48)])
    proj = gs.gs_projected(FAKE, FAKE, FAKE, FAKE)
    bins = gs.gs_bins(FAKE, FAKE, FAKE, FAKE, 100)
    assert lib.gs_render_fwd(ctypes.byref(proj), 10, ctypes.byref(bins), ctypes.byref(v), None,
                             None, FAKE, FAKE, None, None) == 1
    g = _gauss(gs)
    grads = gs.gs_grads(FAKE, FAKE, FAKE, FAKE, FAKE, None)
    need = lib.gs_render_bwd_workspace_size(10, ctypes.byref(v))
    # pose gradient requested but xi is NULL
    assert lib.gs_render_bwd(ctypes.byref(g), ctypes.byref(proj), ctypes.byref(bins), ctypes.byref(v),
                             None, FAKE, FAKE, FAKE, ctypes.byref(grads), 0, FAKE, need, None) == 1
    # exclusive flags, then an unknown flag bit
    grads.xi = FAKE
    assert lib.gs_render_bwd(ctypes.byref(g), ctypes.byref(proj), ctypes.byref(bins), ctypes.byref(v),
                             None, FAKE, FAKE, FAKE, ctypes.byref(grads), 3, FAKE, need, None) == 1
    assert lib.gs_render_bwd(ctypes.byref(g), ctypes.byref(proj), ctypes.byref(bins), ctypes.byref(v),
                             None, FAKE, FAKE, FAKE, ctypes.byref(grads), 16, FAKE, need, None) == 1
    assert lib.gs_render_bwd(ctypes.byref(g), ctypes.byref(proj), ctypes.byref(bins), ctypes.byref(v),
                             None, FAKE, FAKE, FAKE, ctypes.byref(grads), 0, FAKE, need - 1,
                             None) == gs.GS_ERR_CAPACITY


def test_adam_argument_errors(gs):
    lib = gs.lib()
    assert lib.gs_adam_step(FAKE, FAKE, FAKE, FAKE, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None, None) == 1
    assert lib.gs_adam_step(FAKE, FAKE, FAKE, FAKE, 10, 1e-3, 1.0, 0.999, 1e-8, 1, None, None) == 1
    assert lib.gs_adam_step(None, FAKE, FAKE, FAKE, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == 1
    assert lib.gs_adam_step(FAKE, FAKE, FAKE, FAKE, -1, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == 1
    # n == 0 is a no-op that needs no device
    assert lib.gs_adam_step(None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == 0


def test_se3_exp_closed_form_matches_matrix_exponential():
    """Host-side pose update (closed form) vs the matrix exponential."""
    import torch
    from oracle import gs_oracle as O
    from paper_2409_09295_amd.autograd import se3_exp
    rng = np.random.default_rng(0)
    for scale in (1e-12, 1e-3, 0.5, 2.0):
        xi = rng.normal(size=6) * scale
        ref = O.se3_exp(torch.as_tensor(xi)).numpy()
        np.testing.assert_allclose(se3_exp(xi), ref, atol=1e-12)


def _act(gs, c, stride=None, offset=0, n=1, h=8, w=8, data=0xDEAD0000):
    return gs.gs_act(data, n, h, w, c, stride if stride is not None else c, offset)


def test_nn_argument_errors(gs):
    lib = gs.lib()
    bad = gs.GS_ERR_INVALID_ARGUMENT
    ok_x = _act(gs, 32)
    y = _act(gs, 32)
    w = ctypes.c_void_p(0xDEAD1000)
    conv = lambda x1, x2, m, wt, cout, y_: lib.gs_nn_conv3x3(
        ctypes.byref(x1), ctypes.byref(x2) if x2 else None, ctypes.byref(m) if m else None, wt, cout,
        None, 1, ctypes.byref(y_) if y_ else None, None, 0, None)
    assert conv(_act(gs, 12), None, None, w, 32, y) == bad            # channels not a multiple of 8
    assert conv(_act(gs, 32, data=0xDEAD0004), None, None, w, 32, y) == bad   # misaligned
    assert conv(ok_x, _act(gs, 32, h=4), None, w, 32, y) == bad       # concat of different grids
    assert conv(ok_x, None, _act(gs, 16), w, 32, y) == bad            # mask layout
    assert conv(ok_x, None, None, None, 32, y) == bad                 # no weights
    assert conv(ok_x, None, None, ctypes.c_void_p(0xDEAD1002), 32, y) == bad  # misaligned weights
    assert conv(ok_x, None, None, w, 32, None) == bad                 # no output
    assert conv(ok_x, None, None, w, 64, y) == bad                    # y channels != cout
    assert lib.gs_nn_avgpool2(ctypes.byref(_act(gs, 8, h=7)), ctypes.byref(_act(gs, 8, h=3, w=4)),
                              None) == bad
    assert lib.gs_nn_depth_loss(None, None, 1, 8, 8, ctypes.c_float(500.0), None, None, None, None) == bad
    assert lib.gs_cost_volume_workspace_size(1, 64, 64) == 0
    cams = _views(gs, [(64, 48), (64, 48)])
    assert lib.gs_cost_volume_wta(ctypes.c_void_p(0xDEAD0000), ctypes.byref(cams), None,
                                  ctypes.c_void_p(0xDEAD0000), ctypes.c_void_p(0xDEAD0000), 16,
                                  None) == gs.GS_ERR_CAPACITY
    odd = _views(gs, [(64, 48), (66, 48)])
    assert lib.gs_cost_volume_wta(ctypes.c_void_p(0xDEAD0000), ctypes.byref(odd), None,
                                  ctypes.c_void_p(0xDEAD0000), ctypes.c_void_p(0xDEAD0000), 1 << 20,
                                  None) == bad


def test_capacity_error_holds_no_reference_cycle(gs):
    """A caught capacity error must not keep the catching frame's locals
    alive: a step object kept by such a cycle is freed only by a later
    cyclic GC pass, which may run while a graph is being captured."""
    import gc
    import weakref

    class Owner:
        pass

    def raiser():
        raise gs._capacity_error(gs.GS_ERR_CAPACITY, 123)

    def catcher(owner):
        try:
            raiser()
        except gs.GsError as e:
            return e.required

    was = gc.isenabled()
    gc.disable()
    try:
        owner = Owner()
        ref = weakref.ref(owner)
        assert catcher(owner) == 123
        del owner
        assert ref() is None
    finally:
        if was:
            gc.enable()


def test_selective_entry_points_reject_bad_arguments(gs):
    lib = gs.lib()
    bad = gs.GS_ERR_INVALID_ARGUMENT
    v = _views(gs, [(64, 48)])
    proj = gs.gs_projected(FAKE, FAKE, FAKE, FAKE)
    bins = gs.gs_bins(FAKE, FAKE, FAKE, FAKE, 100)
    assert lib.gs_render_error(ctypes.byref(proj), 10, ctypes.byref(bins), ctypes.byref(v), FAKE,
                               None, FAKE, FAKE, None) == bad              # no target
    assert lib.gs_render_error(ctypes.byref(proj), 10, ctypes.byref(bins), ctypes.byref(v), FAKE,
                               FAKE, FAKE, None, None) == bad              # no output
    act = lambda n, views, eps: lib.gs_active_set(FAKE, n, views, ctypes.c_float(eps), None, FAKE,
                                                   None, None, None)
    assert act(10, 0, 1.0) == bad
    assert act(10, 65, 1.0) == bad
    assert act(-1, 1, 1.0) == bad
    assert act(10, 1, float("nan")) == bad
    assert lib.gs_active_set(FAKE, 10, 1, ctypes.c_float(1.0), None, None, None, None, None) == bad
    grp = (gs.gs_adam_group * 2)()
    grp[0] = gs.gs_adam_group(FAKE, FAKE, FAKE, FAKE, 30, 1e-3)
    grp[1] = gs.gs_adam_group(FAKE, FAKE, FAKE, FAKE, 31, 1e-3)   # not a multiple of n_gauss
    masked = lambda n_groups, mask, n_gauss: lib.gs_adam_step_groups_masked_dev(
        grp, n_groups, ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-15), FAKE, mask,
        n_gauss, None, 0, None)
    assert masked(2, FAKE, 10) == bad
    assert masked(1, None, 10) == bad
    assert masked(1, FAKE, 0) == bad


def test_memory_ledger_tracks_current_and_peak(gs):
    """Host-only ledger: per-category current and peak bytes, the overhead
    total without the map, refused over-release, peak reset."""
    lib = gs.lib()
    gs.gs_mem_reset_peaks()
    base = gs.gs_mem_report()
    a = gs.Tracked(gs.GS_MEM_KEYFRAMES, 3 * 640 * 480 * 4)
    b = gs.Tracked(gs.GS_MEM_INIT, 160 * 120 * 64 * 4)
    m = gs.Tracked(gs.GS_MEM_MAP, 1000)
    r = gs.gs_mem_report()
    assert r["current"]["keyframes"] - base["current"]["keyframes"] == 3 * 640 * 480 * 4
    assert r["overhead_current"] - base["overhead_current"] == 3 * 640 * 480 * 4 + 160 * 120 * 64 * 4
    b.release()
    del b
    r2 = gs.gs_mem_report()
    assert r2["overhead_peak"] - base["overhead_current"] == 3 * 640 * 480 * 4 + 160 * 120 * 64 * 4
    assert r2["overhead_current"] - base["overhead_current"] == 3 * 640 * 480 * 4
    assert r2["peak"]["init"] - base["current"]["init"] == 160 * 120 * 64 * 4
    assert lib.gs_mem_track(gs.GS_MEM_POSES, -(r2["current"]["poses"] + 1)) == gs.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_mem_track(99, 1) == gs.GS_ERR_INVALID_ARGUMENT
    del a, m
    gs.gs_mem_reset_peaks()
    r3 = gs.gs_mem_report()
    assert r3["overhead_peak"] == r3["overhead_current"] == base["overhead_current"]


def test_tuning_keys_validate_and_reset(gs):
    """Pixels per lane takes 1, 2 or 4, tile schedules their four
    GS_SCHEDULE_* values and staging batches 1 or 2 splats per thread; 0
    restores each key's default; anything else is rejected and leaves the
    value as it was.  The header's constants match
    the binding's."""
    header = open(os.path.join(ROOT, "include", "gs.h")).read()
    for name in ("GS_TUNE_FWD_SCHEDULE", "GS_TUNE_BWD_SCHEDULE", "GS_SCHEDULE_HEAVIEST_FIRST",
                 "GS_SCHEDULE_TILE_ID", "GS_SCHEDULE_PERSISTENT", "GS_SCHEDULE_PERSISTENT_HALF",
                 "GS_TUNE_FWD_STAGE", "GS_TUNE_BWD_STAGE", "GS_QUEUE_WORDS",
                 "GS_QUEUE_COUNTERS", "GS_QUEUE_STRIDE"):
        m = re.search(rf"\b{name}\s*=\s*(\d+)", header)
        assert m and int(m.group(1)) == getattr(gs, name), name
    try:
        for key in (gs.GS_TUNE_FWD_SCHEDULE, gs.GS_TUNE_BWD_SCHEDULE):
            assert gs.gs_get_tuning(key) == gs.GS_SCHEDULE_HEAVIEST_FIRST
            gs.gs_set_tuning(key, gs.GS_SCHEDULE_PERSISTENT)
            assert gs.gs_get_tuning(key) == gs.GS_SCHEDULE_PERSISTENT
            for bad in (-1, 5, 7):
                with pytest.raises(gs.GsError):
                    gs.gs_set_tuning(key, bad)
            assert gs.gs_get_tuning(key) == gs.GS_SCHEDULE_PERSISTENT
            gs.gs_set_tuning(key, 0)
            assert gs.gs_get_tuning(key) == gs.GS_SCHEDULE_HEAVIEST_FIRST
        for key in (gs.GS_TUNE_FWD_PIXELS_PER_LANE, gs.GS_TUNE_BWD_PIXELS_PER_LANE):
            gs.gs_set_tuning(key, 4)
            with pytest.raises(gs.GsError):
                gs.gs_set_tuning(key, 3)
            assert gs.gs_get_tuning(key) == 4
            gs.gs_set_tuning(key, 0)
            assert gs.gs_get_tuning(key) == 1
        gs.gs_set_tuning(gs.GS_TUNE_FWD_SCHEDULE, gs.GS_SCHEDULE_PERSISTENT_HALF)
        assert gs.gs_get_tuning(gs.GS_TUNE_FWD_SCHEDULE) == gs.GS_SCHEDULE_PERSISTENT_HALF
        for key in (gs.GS_TUNE_FWD_STAGE, gs.GS_TUNE_BWD_STAGE):
            assert gs.gs_get_tuning(key) == 0          # the kernels' own default
            gs.gs_set_tuning(key, 2)
            for bad in (-1, 3, 64):
                with pytest.raises(gs.GsError):
                    gs.gs_set_tuning(key, bad)
            assert gs.gs_get_tuning(key) == 2
            gs.gs_set_tuning(key, 0)
            assert gs.gs_get_tuning(key) == 0
        with pytest.raises(gs.GsError):
            gs.gs_set_tuning(gs.GS_TUNE_BWD_STAGE + 1, 1)
        assert gs.gs_get_tuning(99) < 0
    finally:
        for key in range(6):
            gs.gs_set_tuning(key, 0)


def test_binding_constants_match_the_headers(gs):
    """Every enum constant the Python binding re-declares has the header's
    value (the binding marshals these numbers straight into the C ABI)."""
    text = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("gs.h", "gs_nn.h"))
    declared = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(GS_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    defines = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(GS_[A-Z0-9_]+)\s+(\d+)", text)}
    declared.update(defines)
    bound = {k: v for k, v in vars(gs).items() if k.startswith("GS_") and isinstance(v, int)}
    common = sorted(set(declared) & set(bound))
    assert len(common) >= 20, common
    for name in common:
        assert bound[name] == declared[name], (name, bound[name], declared[name])

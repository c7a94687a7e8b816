"""Host logic of the autotuner's choice (no GPU): the fastest setting wins
unless another lies within the tie margin and departs less from the
kernel's defaults (its own staging batch, heaviest-first launches)."""
from paper_2409_09295_amd import autotune as A


def _settings():
    return [(p, st, name) for name in A.SCHEDULES for p in A.CHOICES for st in A.STAGES]


def _table(kernel, times):
    t = {A._label(kernel, *c): 1.0 for c in _settings()}
    t.update({A._label(kernel, *c): v for c, v in times.items()})
    return t


def test_fastest_setting_wins_outside_the_tie_margin():
    t = _table("bwd", {(4, 1, "persistent"): 0.50, (4, 2, "heaviest_first"): 0.52})
    assert A._pick(_settings(), t, "bwd") == (4, 1, "persistent")


def test_ties_resolve_to_the_kernel_defaults():
    # within the margin: the backward's default batch at 4 pixels per lane is 2 splats
    t = _table("bwd", {(4, 1, "heaviest_first"): 0.700, (4, 2, "heaviest_first"): 0.705})
    assert A._pick(_settings(), t, "bwd") == (4, 2, "heaviest_first")
    # the forward's default at 4 pixels per lane is 1 splat; heaviest first beats persistent
    t = _table("fwd", {(4, 1, "persistent"): 0.340, (4, 1, "heaviest_first"): 0.342,
                       (4, 2, "heaviest_first"): 0.341})
    assert A._pick(_settings(), t, "fwd") == (4, 1, "heaviest_first")


def test_ties_prefer_the_faster_among_equally_default_settings():
    t = _table("fwd", {(2, 2, "heaviest_first"): 0.400, (4, 1, "heaviest_first"): 0.401})
    assert A._pick(_settings(), t, "fwd") == (2, 2, "heaviest_first")


def test_default_batches_match_the_library():
    """The tuner's notion of each kernel's default staging batch is the one
    the launch code falls back to when GS_TUNE_*_STAGE is 0."""
    import os
    import re
    csrc = os.path.join(os.path.dirname(A.__file__), "csrc")
    for kernel, src, key in (("fwd", "render_fwd.hip", "GS_TUNE_FWD_STAGE"),
                             ("bwd", "render_bwd.hip", "GS_TUNE_BWD_STAGE")):
        text = open(os.path.join(csrc, src)).read()
        m = re.search(r"stage_per_thread\(tuning\(" + key + r"\),\s*ppl == (\d) \? (\d) : (\d)\)", text)
        assert m, src
        ppl, hit, other = (int(x) for x in m.groups())
        lib = {p: hit if p == ppl else other for p in A.CHOICES}
        assert A.DEFAULT_STAGE[kernel] == lib, (kernel, A.DEFAULT_STAGE[kernel], lib)

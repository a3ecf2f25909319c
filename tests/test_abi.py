"""CPU checks of the C ABI: the library loads, exports every declared symbol,
validates plans, and its host-side level / schedule planner is bit-exact with
the oracle.  No device work."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle as O
import paper_1009_0881_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmf.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:nmf_status|const char \*)\s*(nmf_\w+)\s*\(", text, re.M)))


def test_header_declares_what_the_binding_lists():
    assert declared_symbols() == sorted(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (nmf_\w+)$", out, re.M))
    assert set(declared_symbols()) <= exported


def test_status_strings():
    L = P.lib()
    for code in range(-7, 1):
        assert L.nmf_status_string(code)


@pytest.mark.parametrize("kw,status", [
    (dict(m=100, n=4, h=10, w=11, r=3), -2),             # m != h*w
    (dict(m=100, n=4, h=10, w=10, r=0), -2),             # r < 1
    (dict(m=100, n=4, h=10, w=10, r=65), -2),            # r > 64
    (dict(m=4, n=4, h=2, w=2, r=1, levels=3), -2),       # side 1 cannot be restricted
    (dict(m=256, n=40, h=16, w=16, r=20, levels=3, algo="anls"), -2),   # 4x4 level < r
    (dict(m=100, n=4, h=10, w=10, r=3, algo=7), -1),     # unknown algorithm
    (dict(m=100, n=0, h=10, w=10, r=3), -2),             # n < 1
    (dict(m=100, n=4, h=10, w=10, r=3, tile_cfg=(3, 4)), -1),    # wc not in {1, 2, 4}
    (dict(m=100, n=4, h=10, w=10, r=3, tile_cfg=(2, 8)), -1),    # cf not in {4, 16}
    (dict(m=100, n=4, h=10, w=10, r=3, tile_cfg=(1 | 16 << 8 | 1 << 17)), -1),
    (dict(m=100, n=4, h=10, w=10, r=3, tile_cfg=(1 << 18)), -1),
    (dict(m=256, n=40, h=16, w=16, r=3, levels=2, two_sided=True, prec="bf16"), -1),
    (dict(m=256, n=2, h=16, w=16, r=1, levels=3, two_sided=True), -2),   # 2 -> 1 column, then 1
    (dict(m=256, n=40, h=16, w=16, r=3, levels=2, algo="kl", prec="bf16"), -1),   # KL: FP32
    (dict(m=256, n=40, h=16, w=16, r=3, levels=2, algo="kl", two_sided=True), -1),  # one-sided
    (dict(m=100, n=4, h=10, w=10, r=3, algo=4), -1),     # past NMF_KL
    (dict(m=100, n=12, h=10, w=10, r=3, ntf_k=5), -2),   # NTF: n not a multiple of K
    (dict(m=100, n=12, h=10, w=10, r=3, ntf_k=3, algo="mu"), -1),        # NTF: HALS only
    (dict(m=100, n=12, h=10, w=10, r=3, ntf_k=3, prec="bf16"), -1),      # NTF: FP32 only
    (dict(m=100, n=12, h=10, w=10, r=3, ntf_k=-1), -1),
])
def test_plan_rejects_bad_descriptions(kw, status):
    with pytest.raises(P.NmfError) as e:
        P.Plan(**kw)
    assert e.value.status == status


def test_hals_allows_coarse_levels_smaller_than_r():
    # 16 -> 8 -> 4 with r = 20: HALS/MU stay well defined
    P.Plan(m=256, n=40, h=16, w=16, r=20, levels=3, algo="hals")


@pytest.mark.parametrize("hw", [(16, 16), (112, 92), (256, 256), (17, 33), (48, 48), (5, 7)])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_level_sides_match_oracle(hw, levels):
    h, w = hw
    pl = P.Plan(m=h * w, n=10, h=h, w=w, r=3, levels=levels)
    assert pl.level_sides() == O.level_sides(h, w, levels)


@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
@pytest.mark.parametrize("levels", [1, 2, 3, 4])
@pytest.mark.parametrize("T", [0, 1, 5, 16, 40, 123, 200, 1000])
def test_schedule_matches_oracle(cycle, levels, T):
    pl = P.Plan(m=256 * 256, n=10, h=256, w=256, r=3, levels=levels, cycle=cycle)
    assert pl.schedule(T) == O.schedule(P.CYCLES[cycle], levels, T)


@pytest.mark.parametrize("cycle", ["ni", "vc", "fmg", "wc"])
@pytest.mark.parametrize("levels", [1, 2, 3, 4])
@pytest.mark.parametrize("T", [0, 1, 5, 16, 123])
def test_two_sided_schedule_matches_oracle(cycle, levels, T):
    pl = P.Plan(m=256 * 256, n=64, h=256, w=256, r=3, levels=levels, cycle=cycle, two_sided=True)
    assert pl.schedule(T) == O.schedule(P.CYCLES[cycle], levels, T, 8)


def test_workspace_grows_with_levels_and_algo():
    a = P.Plan(m=10304, n=400, h=112, w=92, r=40, levels=1).workspace_bytes
    b = P.Plan(m=10304, n=400, h=112, w=92, r=40, levels=3).workspace_bytes
    c = P.Plan(m=10304, n=400, h=112, w=92, r=40, levels=3, algo="anls").workspace_bytes
    assert 0 < a < b < c
    assert b % 256 == 0


def test_plan_accepts_every_tile_candidate():
    from paper_1009_0881_amd import tune
    for wc, cf in tune.CANDIDATES:
        pl = P.Plan(m=256, n=40, h=16, w=16, r=20, levels=2, tile_cfg=(wc, cf))
        assert pl.desc.tile_cfg == P.tile(wc, cf) == (wc | cf << 8)


def test_grouped_flag():
    base = dict(m=2304, n=300, h=48, w=48, r=20, levels=3)
    a = P.Plan(**base)
    g = P.Plan(**base, grouped=True)
    t = P.Plan(**base, tile_cfg=(2, 4), grouped=True)
    assert g.desc.tile_cfg == P.TILE_GROUPED == 1 << 16
    assert t.desc.tile_cfg == P.tile(2, 4) | P.TILE_GROUPED
    # fewer C-pass chunks: the partial buffers shrink
    assert g.workspace_bytes < a.workspace_bytes


def test_tune_cache_round_trip(tmp_path):
    from paper_1009_0881_amd import tune
    kw = dict(m=256, n=40, h=16, w=16, r=20, levels=2, algo="hals")
    path = str(tmp_path / "tiles.json")
    assert tune.choose(kw, "solve", path) == 0               # nothing tuned yet
    tune.save_result(path, tune.shape_key(kw, "solve"),
                     {"best": (2, 4), "tile_cfg": P.tile(2, 4), "ms": {"2,4": 1.0}})
    assert tune.choose(kw, "solve", path) == P.tile(2, 4)
    assert tune.choose(kw, "batch", path) == 0               # other context
    assert tune.choose(dict(kw, r=21), "solve", path) == 0   # other shape class

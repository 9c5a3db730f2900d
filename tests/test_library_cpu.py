"""The HIP library on the CPU: it loads, exports every entry point the C
header declares, and validates configurations (no device calls)."""
import os
import re

import pytest

from paper_2004_14887_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2004_14887_amd import _lib
    try:
        return _lib.load()
    except ImportError as e:
        pytest.skip(str(e))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "dclbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(dclbm_[a-z_0-9]+)\s*\(", src))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = declared_entry_points()
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2004_14887_amd import _lib as L
    assert declared_entry_points() == set(L._SIGS)


def test_workspace_bytes_and_validation():
    _lib()
    from paper_2004_14887_amd._lib import DclbmError
    from paper_2004_14887_amd.sim import workspace_bytes

    wl = W.vortex_2level()
    b64, b32, b16 = (workspace_bytes(wl, p) for p in ("fp64", "fp32", "fp16"))
    assert b64 > b32 > b16 > 0
    # two A/B population buffers per level dominate: FP64 D2Q9 = 2 * 9 * 8 bytes per node
    assert b64 >= 2 * 9 * 8 * (128 * 128 + 129 * 129)
    bad = W.vortex_2level()
    bad.boxes = [((1, 32), (96, 96))]
    with pytest.raises(DclbmError) as ei:
        workspace_bytes(bad)
    assert "margin" in str(ei.value)
    bad.boxes = [((32, 32), (34, 96))]
    with pytest.raises(DclbmError):
        workspace_bytes(bad)
    bad = W.vortex_2level()
    bad.tau0 = 0.5
    with pytest.raises(DclbmError):
        workspace_bytes(bad)
    # the storage reference velocity must be subsonic (and is ignored by FP64)
    with pytest.raises(DclbmError) as ei:
        workspace_bytes(wl, "fp32", u_ref=(0.6, 0.0))
    assert "u_ref" in str(ei.value)
    assert workspace_bytes(wl, "fp32", u_ref=(0.1, 0.05)) == b32


def test_lattice_table_matches_paper_numbering():
    _lib()
    from paper_2004_14887_amd.sim import lattice_table
    xi, w = lattice_table("D2Q9")
    # Fig. 1 labels: 1 E, 2 NE, 3 N, 4 NW, 5 W, 6 SW, 7 S, 8 SE
    assert [v[:2] for v in xi] == [(0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    assert abs(sum(w) - 1) < 1e-15
    xi3, w3 = lattice_table("D3Q19")
    assert len(xi3) == 19 and abs(sum(w3) - 1) < 1e-15


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2004_14887_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "dclbm_oracle" not in text and "liboracle" not in text, f


def test_server_workspace_bytes_and_validation():
    lib = _lib()
    import ctypes as C

    from paper_2004_14887_amd import _lib as L
    from paper_2004_14887_amd.server import server_config

    def total(arena, **kw):
        out = C.c_size_t()
        st = lib.dclbm_server_workspace_bytes(C.byref(server_config(**kw)), arena, C.byref(out))
        return st, out.value

    st, t0 = total(0)
    assert st == 0 and t0 > 0
    st, t1 = total(1 << 30)
    assert st == 0 and t1 - t0 == 1 << 30
    # tables grow with slots and with the phases of deeper meshes (2^L - 1 per step)
    assert total(0, max_slots=128)[1] > t0
    assert total(0, max_levels=4)[1] > total(0, max_levels=2)[1]
    for bad in (dict(max_slots=0), dict(max_levels=5), dict(steps_per_tick=0), dict(grid=12),
                dict(max_probes=33), dict(max_probe_steps=0)):
        st, _ = total(0, **bad)
        assert st == -1, bad
    assert L.REQ_STATE[2] == "done"


def test_checkpoint_entry_points_reject_null_arguments():
    import ctypes as C
    lib = _lib()
    n = C.c_size_t(7)
    assert lib.dclbm_checkpoint_bytes(None, C.byref(n)) == -1 and n.value == 7
    assert lib.dclbm_save(None, None, 0) == -1
    assert lib.dclbm_load(None, None, 0) == -1
    assert "null" in lib.dclbm_last_error().decode()


def test_probe_sum_and_layout_entry_points_reject_null_arguments():
    import ctypes as C
    lib = _lib()
    n = C.c_int64(7)
    assert lib.dclbm_set_probe_window(None, 0, 1) == -1
    assert lib.dclbm_read_probe_sums(None, None, C.byref(n)) == -1 and n.value == 7
    assert lib.dclbm_set_split(None, 0) == -1
    assert "null" in lib.dclbm_last_error().decode()


def test_hrr_configuration_validation():
    _lib()
    from paper_2004_14887_amd._lib import DclbmError
    from paper_2004_14887_amd.sim import workspace_bytes

    wl = W.Workload("h", "D3Q19", (16, 16, 16), [], 0.55, 1, collision="hrr")
    assert workspace_bytes(wl, "fp32") > workspace_bytes(W.Workload("b", "D3Q19", (16, 16, 16), [], 0.55, 1), "fp32")
    # refined meshes carry per-level macroscopic fields, their ring and the
    # co-located nodes' gradients on top of the BGK workspace
    refined = W.vortex_2level(n0=64)
    bgk_bytes = workspace_bytes(refined, "fp32")
    refined.collision = "hrr"
    assert workspace_bytes(refined, "fp32") > bgk_bytes
    wl.hrr_sigma = 1.5
    with pytest.raises(DclbmError):
        workspace_bytes(wl)


def test_region_and_layer_validation():
    """Refined regions: D2Q9, two levels, non-empty; absorbing layers: within
    half the domain, strength in [0, 1], outside the level-1 box."""
    _lib()
    import numpy as np
    from paper_2004_14887_amd._lib import DclbmError
    from paper_2004_14887_amd.sim import workspace_bytes

    wl = W.Workload("r", "D2Q9", (64, 64), [((12, 12), (52, 52))], 0.55, 1)
    wl.region = W.circle_region(wl.boxes[0], (32.0, 32.0), 16.0)
    assert workspace_bytes(wl, "fp32") > 0
    empty = W.Workload("r", "D2Q9", (64, 64), [((12, 12), (52, 52))], 0.55, 1)
    empty.region = np.zeros((40, 40), np.uint8)
    three = W.Workload("r", "D2Q9", (64, 64), [((12, 12), (52, 52)), ((10, 10), (30, 30))], 0.55, 1)
    three.region = wl.region
    for bad in (empty, three):
        with pytest.raises(DclbmError):
            workspace_bytes(bad, "fp32")
    lay = W.Workload("s", "D2Q9", (64, 64), [((16, 16), (48, 48))], 0.55, 1, sponge_cells=12, sponge_sigma=0.3)
    assert workspace_bytes(lay, "fp32") > 0
    for cells, sigma in ((17, 0.3), (33, 0.3), (12, 1.5)):
        lay.sponge_cells, lay.sponge_sigma = cells, sigma
        with pytest.raises(DclbmError):
            workspace_bytes(lay, "fp32")

"""The project autotuner: picks a valid launch shape, caches it per device
architecture, and the chosen shape keeps parity with the oracle."""
import json

import pytest
import torch

from _parity import compare_state, gpu_run, log, oracle_run
from paper_0911_5692_amd import autotune
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_cache_and_parity(tmp_path):
    w = W.CFG2.resized(48)
    cache = str(tmp_path / "tune.jsonl")
    first = autotune(**w.model(), dtype=torch.float32, cache_path=cache)
    log(f"[tune] {first}")
    assert first["ms"] > 0
    assert first["tile_y"] in (1, 4, 8, 16)
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1 and lines[0]["N"] == 48 and lines[0]["arch"].startswith("gfx")
    again = autotune(**w.model(), dtype=torch.float32, cache_path=cache)
    assert again["ms"] == -1.0
    assert {k: again[k] for k in ("tile_x", "tile_y", "zchunk")} == \
        {k: first[k] for k in ("tile_x", "tile_y", "zchunk")}
    st, _, _, ic = oracle_run(w, 80)
    lat, _ = gpu_run(w, ic, 80, tile_x=first["tile_x"], tile_y=first["tile_y"], zchunk=first["zchunk"])
    errs = compare_state([x.cpu().numpy() for x in lat.fields(dtype=torch.float64)], st)
    assert max(errs.values()) <= 1e-5, errs


def test_lattice_takes_the_tuned_shape(tmp_path):
    """Lattice(..., tuned=path) uses the cached choice; an explicit shape wins."""
    from paper_0911_5692_amd import Lattice
    w = W.CFG2.resized(40)
    cache = str(tmp_path / "tune.jsonl")
    best = autotune(**w.model(), dtype=torch.float32, cache_path=cache)
    lat = Lattice(**w.model(), dtype=torch.float32, tuned=cache)
    assert lat.launch_shape == {k: best[k] for k in ("tile_x", "tile_y", "zchunk")}
    lat.close()
    lat = Lattice(**w.model(), dtype=torch.float32, tuned=cache, tile_x=64, tile_y=4, zchunk=8)
    assert lat.launch_shape == dict(tile_x=64, tile_y=4, zchunk=8)
    lat.close()

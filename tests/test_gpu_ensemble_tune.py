"""The ensemble autotuner and the 32-wide tiles it can choose.

The tuner picks a tile and a target z-chunk by timing the batched sweep of
the given realizations, caches the choice per device architecture and
multiset of lattice sizes, and the tuned ensemble keeps parity with the
oracle.  32-wide tiles (which split 96^3 and 160^3 rows without a ragged
tile) give each realization bitwise the state of a lone lattice run with the
same tile, and the oracle's within the FP32 bar."""
import json

import pytest
import torch

from _parity import compare_state, log, oracle_run, to_dev
from paper_0911_5692_amd import Ensemble, Lattice, ens_autotune
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu


def _init(ens, members):
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        ens.init_physical(r, *(to_dev(ic[k]) for k in ("f1", "f2", "u1", "u2")), ic["a0"])


def test_ensemble_autotune_cache_and_parity(tmp_path):
    members = [W.CFG1.resized(n) for n in (16, 24, 40, 33, 16, 48)]
    models = [m.model() for m in members]
    cache = str(tmp_path / "tune.jsonl")
    first = ens_autotune(models, torch.float32, cache_path=cache)
    log(f"[ens-tune] {first}")
    assert first["ms"] > 0 and first["tile_x"] in (32, 64, 128) and first["tile_y"] in (4, 8, 16)
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1 and lines[0]["ensemble"] == "16:2,24:1,33:1,40:1,48:1"
    again = ens_autotune(models, torch.float32, cache_path=cache)
    assert again["ms"] == -1.0
    assert {k: again[k] for k in ("tile_x", "tile_y", "ztarget", "zchunks")} == \
        {k: first[k] for k in ("tile_x", "tile_y", "ztarget", "zchunks")}
    ens = Ensemble(models, dtype=torch.float32, tuned=cache)
    assert ens.tuning["ms"] == -1.0
    _init(ens, members)
    steps = 60
    ens.step(steps)
    for r, m in enumerate(members):
        st, oe, _, _ = oracle_run(m, steps, realization=r)
        errs = compare_state([x.cpu().numpy() for x in ens.fields(r)], st)
        assert max(errs.values()) <= 1e-5, (r, errs)
    ens.close()


@pytest.mark.parametrize("tile_y", [8, 16])
def test_32_wide_tiles_bitwise_lone_and_oracle(tile_y):
    members = [W.CFG1.resized(n) for n in (32, 96, 40, 20)]
    zchunks = [16, 48, 40, 7]
    ens = Ensemble([m.model() for m in members], dtype=torch.float32, tile_x=32, tile_y=tile_y, zchunks=zchunks)
    _init(ens, members)
    n = 33
    ens.step(n)
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        lat = Lattice(**m.model(), dtype=torch.float32, tile_x=32, tile_y=tile_y, zchunk=zchunks[r])
        lat.init_physical(*(to_dev(ic[k]) for k in ("f1", "f2", "u1", "u2")), ic["a0"])
        lat.step(n)
        for x, y in zip(ens.fields(r), lat.fields()):
            assert torch.equal(x, y), r
        assert ens.energies()[r] == lat.energies()
        lat.close()
        st, _, _, _ = oracle_run(m, n, realization=r)
        errs = compare_state([x.cpu().numpy() for x in ens.fields(r)], st)
        log(f"[ens32] tile 32x{tile_y} r={r} N={m.N}: {errs}")
        assert max(errs.values()) <= 1e-5, (r, errs)
    ens.close()


def test_32_wide_tile_rejected_for_27_points():
    from dataclasses import replace
    from paper_0911_5692_amd import LfError
    m = replace(W.CFG1.resized(32), stencil=27)
    with pytest.raises(LfError) as ei:
        Lattice(**m.model(), dtype=torch.float32, tile_x=32, tile_y=8)
    assert ei.value.code == 1

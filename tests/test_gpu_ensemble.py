"""The batched ensemble path of liblf: uneven realizations in one persistent,
graph-captured launch per step, against the FP64 oracle and against
single-lattice runs."""
import numpy as np
import pytest
import torch

from _parity import ARRAYS, compare_state, log, oracle_run, to_dev
from paper_0911_5692_amd import Ensemble, Lattice
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu


def _build(members, dtype, **kw):
    ens = Ensemble([m.model() for m in members], dtype=dtype, **kw)
    ad0s = []
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        ad0s.append(ens.init_physical(r, *(to_dev(ic[k]) for k in ("f1", "f2", "u1", "u2")), ic["a0"]))
    return ens, ad0s


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-10)])
def test_mixed_ensemble_matches_oracle(dtype, tol):
    sizes = [16, 16, 24, 40, 16, 24, 33]
    members = [W.CFG1.resized(n) for n in sizes]
    steps = 90
    ens, ad0s = _build(members, dtype)
    ens.step(steps)
    en = ens.energies()
    for r, m in enumerate(members):
        st, oe, oad0, _ = oracle_run(m, steps, realization=r)
        assert abs(ad0s[r] - oad0) <= 1e-12 * oad0
        errs = compare_state([x.cpu().numpy() for x in ens.fields(r)], st)
        log(f"[ens] r={r} N={m.N} {errs}")
        assert max(errs.values()) <= tol, (r, errs)
        assert abs(en[r]["a"] - oe["a"]) <= (1e-12 if dtype == torch.float64 else 1e-9) * oe["a"]
        assert en[r]["step"] == steps


def test_ensemble_equals_single_lattice_bitwise():
    """Same tile and z-chunk: a realization of the ensemble and a lone lattice
    do the same arithmetic in the same order."""
    members = [W.CFG1.resized(n) for n in (32, 48, 20)]
    ens, _ = _build(members, torch.float32, tile_x=64, tile_y=8, zchunks=[16, 16, 16])
    n = 41
    ens.step(n)
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        lat = Lattice(**m.model(), dtype=torch.float32, tile_x=64, tile_y=8, zchunk=16)
        lat.init_physical(*(to_dev(ic[k]) for k in ("f1", "f2", "u1", "u2")), ic["a0"])
        lat.step(n)
        a = ens.fields(r)
        b = lat.fields()
        for x, y in zip(a, b):
            assert torch.equal(x, y), r
        assert ens.energies()[r] == lat.energies()


def test_workload4_full_ensemble_sampled():
    """48 x 64^3 + 16 x 96^3 + 4 x 160^3, 500 steps, one launch per step:
    realizations sampled from each size class against the oracle."""
    members = W.ensemble_members()
    steps = W.ENSEMBLE_STEPS
    log(f"[ens] building {len(members)} realizations")
    ens, ad0s = _build(members, torch.float32)
    ens.step(steps)
    torch.cuda.synchronize()
    log(f"[ens] {steps} steps in {ens.last_step_ms():.1f} ms")
    en = ens.energies()
    assert all(e["step"] == steps and e["status"] == 0 for e in en)
    for r in (0, 47, 48, 67):
        st, oe, _, _ = oracle_run(members[r], steps, realization=r)
        errs = compare_state([x.cpu().numpy() for x in ens.fields(r)], st)
        log(f"[ens] r={r} N={members[r].N}: {errs}")
        assert max(errs.values()) <= 1e-5, (r, errs)
        assert abs(en[r]["a"] - oe["a"]) <= 1e-9 * oe["a"]

"""The budget observed, not planned: every query here runs in a caller-owned workspace
of exactly the budget, with guard bands of a known pattern on both sides, and the
bands must be intact afterwards -- no kernel of any engine wrote outside the budget.
(The pool_high_water statistic is the planner's own figure; this checks the memory.)
"""
import numpy as np
import pytest

from datagen import workloads
from tests.gpu_util import check_against_oracle, lib_spec_args
from tests.wl import oracle_spec

pytestmark = pytest.mark.gpu
MIB = 1 << 20
GUARD = 4 * MIB


def _run_guarded(rec, wl, budget, **kw):
    import torch
    import paper_1311_0059_amd as P

    raw = torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1).copy()).cuda()
    slab = torch.empty(GUARD + budget + GUARD, dtype=torch.uint8, device="cuda")
    pattern = torch.arange(slab.numel(), device="cuda", dtype=torch.int64).remainder(251).to(torch.uint8)
    slab.copy_(pattern)
    torch.cuda.synchronize()
    ws = slab[GUARD:GUARD + budget]
    spec = P.make_spec(wl.record_bytes, list(wl.key_fields), list(wl.aggs), budget=budget, workspace=ws, **kw)
    with P.GroupBy(spec) as g:
        g.consume_ptr(raw.data_ptr(), rec.size)
        g.finish()
        k, c = g.rows("cpu")
        st = g.stats()
    torch.cuda.synchronize()
    lo_ok = torch.equal(slab[:GUARD], pattern[:GUARD])
    hi_ok = torch.equal(slab[GUARD + budget:], pattern[GUARD + budget:])
    keys = k.numpy().view(np.uint64)
    order = np.argsort(keys, kind="stable")
    return keys[order], c.numpy()[:, order], st, lo_ok, hi_ok


@pytest.mark.parametrize("engine,policy,budget_mib", [("auto", "destage", 8), ("lds", "destage", 3),
                                                      ("tables", "destage", 3), ("tables", "prepart", 3),
                                                      ("owner", "destage", 8), ("onchip", "destage", 4),
                                                      ("tables", "hashsort", 2)])
def test_no_write_outside_the_budget(engine, policy, budget_mib):
    wl = workloads.uniform_spill().scaled(1_500_000, 300_000)
    if engine == "onchip":
        wl = workloads.uniform_small().scaled(2_000_000, 8_000)
    rec = wl.generate()
    print(f"case: budget guard {engine} {policy} {budget_mib}MiB", flush=True)
    k, c, st, lo_ok, hi_ok = _run_guarded(rec, wl, budget_mib * MIB, est_groups=wl.d, engine=engine, policy=policy)
    check_against_oracle(rec, oracle_spec(wl), k, c, f"guard {engine} {policy}")
    assert lo_ok and hi_ok, "a kernel wrote outside the workspace"

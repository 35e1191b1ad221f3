"""The entry point that allocates nothing (agg_query_noalloc) against the
existing path (agg_create / agg_consume / agg_finish), through the C ABI.

Two calls in a row, the second with a smaller input, so that the second call's
rows show that it cleared what the first left in the device array; then the
errors: too many groups for the array's table, too small an output.
"""
import numpy as np
import pytest

from datagen import workloads
from tests.gpu_util import assert_rows_equal, lib_spec_args, run_lib

pytestmark = pytest.mark.gpu


def _noalloc(rec, wl, est, cap=None):
    import torch
    import paper_1311_0059_amd as P
    dev = torch.from_numpy(rec.view(np.uint8).reshape(-1).copy()).to("cuda")
    cap = wl.n if cap is None else cap
    keys = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
    cols = torch.empty((len(wl.aggs), max(cap, 1)), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    spec = P.make_spec(wl.record_bytes, wl.key_fields, wl.aggs, est_groups=est)
    rows = P.query_noalloc(spec, dev.data_ptr(), wl.n, keys, cols)
    k = keys[:rows].cpu().numpy().view(np.uint64)
    c = cols[:, :rows].cpu().numpy()
    o = np.argsort(k, kind="stable")
    return k[o], c[:, o]


@pytest.mark.parametrize("first,second", [((1_000_000, 10_000), (50_000, 2_000)),
                                          ((400_000, 20_000), (3_000, 2_900))])
def test_two_calls_equal_the_query_path(first, second):
    for i, (n, d) in enumerate((first, second)):
        wl = workloads.uniform_small().scaled(n, d)
        rec = wl.generate()
        print(f"case: noalloc call {i} n={n} d={d}", flush=True)
        k, c = _noalloc(rec, wl, d)
        wk, wc, st = run_lib(rec, **lib_spec_args(wl), est_groups=d)
        assert k.size == d
        assert_rows_equal(k, c, wk, wc, f"noalloc call {i}")


def test_r24_and_reserved_keys():
    wl = workloads.zipf_composite().scaled(300_000, 5_000)
    rec = wl.generate().copy()
    rec["k1"][::1001] = 0xFFFFFFFF
    rec["k2"][::1001] = 0xFFFFFFFF  # the all-ones key: a side group
    print("case: noalloc R24", flush=True)
    k, c = _noalloc(rec, wl, 5_001)
    wk, wc, _ = run_lib(rec, **lib_spec_args(wl), est_groups=5_001)
    assert_rows_equal(k, c, wk, wc, "noalloc R24")


def test_r16_reserved_keys_several_classes():
    """16-byte records with reserved key values and more groups than one LDS table: the
    entry point runs the general kernel (the side groups), the rows equal the query path's."""
    wl = workloads.uniform_small().scaled(400_000, 9_000)
    rec = wl.generate().copy()
    rec["key"][::997] = np.uint64(2**64 - 1)
    rec["key"][3::991] = np.uint64(2**64 - 2)
    print("case: noalloc R16 reserved keys", flush=True)
    k, c = _noalloc(rec, wl, 9_002)
    wk, wc, _ = run_lib(rec, **lib_spec_args(wl), est_groups=9_002)
    assert_rows_equal(k, c, wk, wc, "noalloc R16 reserved")


def test_errors():
    import paper_1311_0059_amd as P
    wl = workloads.uniform_small().scaled(200_000, 60_000)
    rec = wl.generate()
    print("case: noalloc too many groups", flush=True)
    with pytest.raises(P.AggError) as e:  # the estimate exceeds what the device array holds
        _noalloc(rec, wl, 60_000)
    assert e.value.status == -2
    wl = workloads.uniform_small().scaled(200_000, 150_000)
    with pytest.raises(P.AggError) as e:  # the estimate is low: the groups found exceed the table
        _noalloc(wl.generate(), wl, 5_000)
    assert e.value.status == -2
    wl = workloads.uniform_small().scaled(100_000, 3_000)
    print("case: noalloc output too small", flush=True)
    with pytest.raises(P.AggError) as e:
        _noalloc(wl.generate(), wl, 3_000, cap=100)
    assert e.value.status == -1 and e.value.rows == 3_000

"""Pins for the CPU oracle: everything here checks it against something other
than itself -- a brute-force group-by, closed forms on constructed inputs, the
paper's special datasets (heavy hitter, all-unique, single key, sorted input),
whole-result invariants, and planted mistakes that the pins must catch.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import datagen
import oracle
from datagen import workloads
from tests.wl import brute_force, make_spec, oracle_spec

EDGE_U64 = [0, 1, (1 << 63) - 1, 1 << 63, (1 << 64) - 2, (1 << 64) - 1]
EDGE_I64 = [-(1 << 63), -1, 0, 1, (1 << 63) - 1]
EDGE_I32 = [-(1 << 31), -1, 0, 1, (1 << 31) - 1]
EDGE_U32 = [0, 1, (1 << 31), (1 << 32) - 1]

SPEC_R16 = make_spec(16, [(0, "u64")], workloads.AGGS_R16_ALL)
SPEC_R24 = make_spec(24, [(0, "u32"), (4, "u32")], workloads.AGGS_R24)
# a layout mixing unsigned inputs: {u32 key @0, u32 a @4, u64 b @8}
SPEC_MIX = make_spec(16, [(0, "u32")], [("MIN", 4, "u32"), ("MAX", 4, "u32"), ("MIN", 8, "u64"), ("MAX", 8, "u64"),
                                         ("SUM", 4, "u32"), ("COUNT", 0, "u32")])
MIX = np.dtype([("key", "<u4"), ("a", "<u4"), ("b", "<u8")])


def _rand_r16(rng, n, pool):
    rec = np.empty(n, dtype=datagen.R16)
    rec["key"] = rng.choice(np.array(pool, dtype=np.uint64), size=n)
    vals = np.concatenate([np.array(EDGE_I64, dtype=np.int64), rng.integers(-50, 50, size=8)])
    rec["v"] = rng.choice(vals, size=n)
    return rec


def _rand_r24(rng, n, pool):
    rec = np.empty(n, dtype=datagen.R24)
    k = rng.choice(np.array(pool, dtype=np.uint64), size=n)
    rec["k1"] = (k >> np.uint64(32)).astype(np.uint32)
    rec["k2"] = (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    rec["v1"] = rng.choice(np.array(EDGE_I64 + [5, -7], dtype=np.int64), size=n)
    rec["v2"] = rng.choice(np.array(EDGE_I32 + [3], dtype=np.int32), size=n)
    rec["v3"] = rng.choice(np.array(EDGE_I32 + [-3], dtype=np.int32), size=n)
    return rec


def _rand_mix(rng, n, pool):
    rec = np.empty(n, dtype=MIX)
    rec["key"] = rng.choice(np.array([p & 0xFFFFFFFF for p in pool], dtype=np.uint32), size=n)
    rec["a"] = rng.choice(np.array(EDGE_U32 + [77], dtype=np.uint32), size=n)
    rec["b"] = rng.choice(np.array(EDGE_U64 + [12345], dtype=np.uint64), size=n)
    return rec


def _pool(rng, size):
    extra = [int(x) for x in rng.integers(0, 1 << 63, size=size, dtype=np.int64)]
    pool = EDGE_U64 + [(1 << 32) - 1, 1 << 32, ((1 << 32) + 5)] + extra
    return pool[: max(1, size)]


def _same(a, b):
    ka, ca = a
    kb, cb = b
    return ka.shape == kb.shape and np.array_equal(ka, kb) and np.array_equal(ca, cb)


BRUTE_CASES = 3400  # per layout: 10,200 tiny inputs in all


def _par(rec, spec, rng):
    """The parallel path with a random thread count and digit width (many buckets on tiny inputs)."""
    return oracle.groupby_par(rec, spec, threads=int(rng.integers(1, 6)), bits=int(rng.integers(1, 17)))


@pytest.mark.parametrize("layout", ["R16", "R24", "MIX"])
def test_oracle_matches_brute_force(layout):
    """Many tiny seeded inputs with keys and values at the edges of their types, through both the
    single-threaded oracle and its parallel form."""
    rng = np.random.default_rng(1311 + len(layout))
    gen, spec = {"R16": (_rand_r16, SPEC_R16), "R24": (_rand_r24, SPEC_R24), "MIX": (_rand_mix, SPEC_MIX)}[layout]
    for case in range(BRUTE_CASES):
        n = int(rng.integers(0, 120 if case % 10 else 1200))
        pool = _pool(rng, int(rng.integers(1, 50)))
        rec = gen(rng, n, pool)
        want = brute_force(rec, spec)
        assert _same(oracle.groupby(rec, spec), want), f"case {case} n={n}"
        assert _same(_par(rec, spec, rng), want), f"case {case} n={n} (parallel)"


def test_parallel_oracle_on_workloads():
    """The parallel form gives the single-threaded oracle's rows on generated workloads, for
    several thread counts and digit widths, and rejects invalid arguments."""
    for wl in (workloads.uniform_small().scaled(300_000, 20_000), workloads.zipf_composite().scaled(300_000, 30_000),
               workloads.heavy_hitter(50_000, 300)):
        rec = wl.generate()
        spec = oracle_spec(wl)
        want = oracle.groupby(rec, spec)
        for threads, bits in ((1, 1), (2, 7), (7, 12), (16, 16)):
            assert _same(oracle.groupby_par(rec, spec, threads=threads, bits=bits), want), (wl.name, threads, bits)
    rec = datagen.r16(5, 100, 10)
    for threads, bits in ((0, 8), (4, 0), (4, 17)):
        with pytest.raises(ValueError):
            oracle.groupby_par(rec, SPEC_R16, threads=threads, bits=bits)
    assert oracle.groupby_par(np.empty(0, dtype=datagen.R16), SPEC_R16)[0].size == 0


def test_empty_input_gives_no_rows():
    rec = np.empty(0, dtype=datagen.R16)
    keys, cols = oracle.groupby(rec, SPEC_R16)
    assert keys.size == 0 and cols.shape == (4, 0)


def test_closed_form_counts_and_ranges():
    """Key i appears c_i times with values 0..c_i-1: COUNT=c_i, SUM=c_i(c_i-1)/2, MIN=0, MAX=c_i-1."""
    rng = np.random.default_rng(7)
    c = rng.integers(1, 60, size=300)
    keys = rng.permutation(np.arange(300, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15))
    rec = np.empty(int(c.sum()), dtype=datagen.R16)
    rec["key"] = np.repeat(keys, c)
    rec["v"] = np.concatenate([np.arange(ci) for ci in c])
    perm = rng.permutation(rec.size)
    rec = rec[perm]
    k, cols = oracle.groupby(rec, SPEC_R16)
    order = np.argsort(keys)
    cs = c[order]
    assert np.array_equal(k, np.sort(keys))
    assert np.array_equal(cols[0], cs)
    assert np.array_equal(cols[1], cs * (cs - 1) // 2)
    assert np.all(cols[2] == 0)
    assert np.array_equal(cols[3], cs - 1)


def test_sum_wraps_modulo_2_64():
    rec = np.zeros(3, dtype=datagen.R16)
    rec["key"] = 42
    rec["v"] = [(1 << 63) - 1, 1, 5]
    _, cols = oracle.groupby(rec, SPEC_R16)
    assert cols[1, 0] == -(1 << 63) + 5
    assert cols[2, 0] == 1 and cols[3, 0] == (1 << 63) - 1


def test_heavy_hitter_closed_form():
    """The paper's heavy-hitter set (Sec. 6.4, "Aggregating Skewed Data"): one key gets n-(d-1) records, all others one each."""
    wl = workloads.heavy_hitter(20_000, 500)
    rec = wl.generate()
    k, cols = oracle.groupby(rec, oracle_spec(wl))
    assert k.size == 500
    counts = np.sort(cols[0])
    assert counts[-1] == 20_000 - 499 and np.all(counts[:-1] == 1)
    single = cols[0] == 1
    assert np.array_equal(cols[1][single], cols[2][single]) and np.array_equal(cols[2][single], cols[3][single])


def test_all_unique_and_single_key():
    """100% cardinality ratio: every row has COUNT 1; one key: one row equal to the global aggregates."""
    rng = np.random.default_rng(3)
    rec = np.empty(5000, dtype=datagen.R16)
    rec["key"] = rng.permutation(np.arange(5000, dtype=np.uint64) * np.uint64(3) + np.uint64(11))
    rec["v"] = rng.integers(-10**12, 10**12, size=5000)
    k, cols = oracle.groupby(rec, SPEC_R16)
    assert k.size == 5000 and np.all(cols[0] == 1)
    assert np.array_equal(cols[1], cols[2]) and np.array_equal(cols[2], cols[3])
    rec["key"] = (1 << 64) - 1
    k, cols = oracle.groupby(rec, SPEC_R16)
    tot = oracle.totals(rec, SPEC_R16)
    assert k.tolist() == [(1 << 64) - 1]
    assert cols[:, 0].tolist() == [5000, int(np.sum(rec["v"])), int(rec["v"].min()), int(rec["v"].max())]
    assert cols[:, 0].tolist() == tot.tolist()


def test_sorted_input_equals_unsorted():
    """The paper's sorted-uniform set (Sec. 6.4) holds the same rows as its unsorted permutation."""
    rec = datagen.r16(99, 50_000, 2_000)
    srt = rec[np.argsort(rec["key"], kind="stable")]
    a = oracle.groupby(rec, SPEC_R16)
    b = oracle.groupby(srt, SPEC_R16)
    assert _same(a, b)


def test_invariants_on_small_workload():
    """The 1M-record / 10k-key workload: rows = D, sum COUNT = N, wrap-around sum, global min / max."""
    wl = workloads.uniform_small()
    rec = wl.generate()
    spec = oracle_spec(wl)
    k, cols = oracle.groupby(rec, spec)
    assert k.size == wl.d
    assert np.all(np.diff(k.astype(np.uint64)) > 0)
    assert cols[0].sum() == wl.n
    assert int(cols[1].astype(np.uint64).sum(dtype=np.uint64)) == int(rec["v"].astype(np.uint64).sum(dtype=np.uint64))
    assert cols[2].min() == rec["v"].min() and cols[3].max() == rec["v"].max()
    assert np.all(cols[0] >= 1) and np.all(cols[2] <= cols[3])


def test_invariants_composite_zipf():
    wl = workloads.zipf_composite().scaled(400_000, 40_000)
    rec = wl.generate()
    spec = oracle_spec(wl)
    k, cols = oracle.groupby(rec, spec)
    assert k.size == wl.d
    sums = cols[0].astype(np.uint64).sum(dtype=np.uint64)
    assert int(sums) == int(rec["v1"].astype(np.uint64).sum(dtype=np.uint64))
    assert cols[1].min() == rec["v2"].min() and cols[2].max() == rec["v3"].max()
    assert cols[3].sum() == wl.n
    # composite order is (k1, k2) lexicographic
    k1, k2 = k >> np.uint64(32), k & np.uint64(0xFFFFFFFF)
    lex = np.lexsort((k2, k1))
    assert np.array_equal(lex, np.arange(k.size))


def test_rows_for_keys_matches_groupby():
    wl = workloads.uniform_small().scaled(200_000, 3_000)
    rec = wl.generate()
    spec = oracle_spec(wl)
    k, cols = oracle.groupby(rec, spec)
    pick = np.random.default_rng(5).choice(k.size, size=64, replace=False)
    q, found, qc = oracle.rows_for_keys(rec, spec, k[pick])
    idx = np.searchsorted(k, q)
    assert np.array_equal(found.astype(np.int64), cols[0, idx])
    assert np.array_equal(qc, cols[:, idx])
    q2, f2, _ = oracle.rows_for_keys(rec, spec, [12345])  # absent key
    assert f2.tolist() == [0] or q2[0] in k


def test_yao_formulas_against_exact_and_simulation():
    """Appendix, input component: Yao's I_key against the exact hypergeometric expectation and a
    simulation of draws without replacement; I_raw is its inverse in r."""
    from math import comb
    n, m = 1200, 60
    per = n // m
    rng = np.random.default_rng(11)
    pool = np.repeat(np.arange(m), per)
    for r in (10, 60, 300, 900):
        exact = m * (1 - comb(n - per, r) / comb(n, r))
        assert abs(oracle.yao_i_key(r, n, m) - exact) / exact < 0.02
        sim = np.mean([np.unique(rng.permutation(pool)[:r]).size for _ in range(400)])
        assert abs(oracle.yao_i_key(r, n, m) - sim) / sim < 0.03
    for k in (5, 30, 55):
        r = oracle.yao_i_raw(k, n, m)
        assert abs(oracle.yao_i_key(r, n, m) - k) < 1e-6
        draws = []
        for _ in range(300):
            seen, cnt = set(), 0
            for x in rng.permutation(pool):
                cnt += 1
                seen.add(int(x))
                if len(seen) == k:
                    break
            draws.append(cnt)
        assert abs(np.mean(draws) - r) / r < 0.1


def test_formula_one_partitions_cover_the_groups():
    """Sec. 4.3, Formula (1): the resident part (M-P frames) plus P spilled partitions of at most
    M-1 frames each must hold G*F frames; P = 0 exactly when everything fits in memory."""
    for G in (1, 10, 100, 1000, 12345, 10**6):
        for M in (3, 4, 16, 100, 4096):
            F = 1.2
            P = oracle.hybrid_hash_partitions(G, M, F)
            if G * F <= M:
                assert P == 0
            else:
                assert (M - P) + (M - 1) * P >= G * F - 1e-9
                if P > 1:  # minimal: one fewer partition does not cover
                    assert (M - (P - 1)) + (M - 1) * (P - 1) < G * F
    with pytest.raises(ValueError):
        oracle.hybrid_hash_partitions(10, 2)


def test_spilled_fraction_against_simulation():
    """Secs. 5.3.1 / 5.3.4: with uniform keys and K of the G_t groups resident, the records spilled
    are R (1 - K / G_t).  Checked against simulated streams in which the first K distinct keys stay
    resident (Pre-Partitioning's partition 0, Sec. 4.3.4) and every record of another key is
    spilled, within 3%, for several K / G_t: keys drawn uniformly with replacement (200 records per
    key, so the keys seen first are barely more frequent than the others), and the dataset D(n, m)
    of the Appendix (every key exactly n / m times, in random order)."""
    rng = np.random.default_rng(53)
    G, N = 5_000, 1_000_000
    streams = (rng.integers(0, G, size=N), rng.permutation(np.repeat(np.arange(G), N // G)))
    for keys in streams:
        first_seen = np.full(G, N)
        np.minimum.at(first_seen, keys, np.arange(keys.size))
        order = np.argsort(first_seen, kind="stable")
        for frac in (0.1, 0.3, 0.55, 0.8):
            K = int(frac * G)
            resident = np.zeros(G, dtype=bool)
            resident[order[:K]] = True
            spilled = int(np.count_nonzero(~resident[keys]))
            model = keys.size * oracle.spilled_fraction(K, G)
            assert abs(spilled - model) / model < 0.03, (frac, spilled, model)
    assert oracle.spilled_fraction(G, G) == 0.0 and oracle.spilled_fraction(2 * G, G) == 0.0


def test_slot_filter_false_positive_against_simulation():
    """Secs. 4.3.4 / 5.3.4: a one-byte filter per slot, each key setting one of the 8 bits of its home
    slot's byte.  Simulated: K keys with uniform home slots and bits set their bits; absent keys
    (their own uniform home slot and bit) test theirs.  The share that find their bit set matches
    1 - (1 - 1/(8H))^K within 2%, at several loads K/H; also the closed forms at K = 0 and K = 1."""
    rng = np.random.default_rng(59)
    H = 50_000
    for load in (0.3, 0.7, 0.9, 1.5):
        K = int(load * H)
        filt = np.zeros(H, dtype=np.uint8)
        np.bitwise_or.at(filt, rng.integers(0, H, size=K), (1 << rng.integers(0, 8, size=K)).astype(np.uint8))
        q = 400_000
        hit = (filt[rng.integers(0, H, size=q)] & (1 << rng.integers(0, 8, size=q)).astype(np.uint8)) != 0
        model = oracle.slot_filter_false_positive(K, H)
        assert abs(hit.mean() - model) / model < 0.02, (load, hit.mean(), model)
    assert oracle.slot_filter_false_positive(0, H) == 0.0
    assert abs(oracle.slot_filter_false_positive(1, H) - 1.0 / (8 * H)) < 1e-15


# ---- planted mistakes: each mutant of the oracle must fail one of the pins above --------------------

MUTANTS = {
    "min_unsigned": ("return or_signed(type) ? ((int64_t)a < (int64_t)b) : (a < b);", "return a < b;"),
    "drop_last_flush": ("  out_keys[rows] = p[n - 1].key;\n  for (uint32_t a = 0; a < na; ++a) out_cols[a * cap + rows] = (int64_t)acc[a];\n  ++rows;\n  free(p);",
                        "  free(p);"),
    "swap_composite": ("return (hi << 32) | lo;", "return (lo << 32) | hi;"),
    "count_from_zero": ("case OR_COUNT: *acc = first ? 1 : *acc + 1; break;", "case OR_COUNT: *acc = first ? 0 : *acc + 1; break;"),
    "max_as_min": ("case OR_MAX: if (first || or_less(*acc, v, type)) *acc = v; break;",
                   "case OR_MAX: if (first || or_less(v, *acc, type)) *acc = v; break;"),
    "i32_zero_extend": ("case OR_I32: { int32_t x; memcpy(&x, rec + off, 4); return (uint64_t)(int64_t)x; }",
                        "case OR_I32: { uint32_t x; memcpy(&x, rec + off, 4); return (uint64_t)x; }"),
    # mistakes in the parallel form only
    "par_bucket_low_bits": ("static uint64_t or_bucket(uint64_t key, uint32_t bits) { return key >> (64 - bits); }",
                            "static uint64_t or_bucket(uint64_t key, uint32_t bits) { return key & ((1ull << bits) - 1); }"),
    "par_bucket_start_late": ("      at += cnt;\n    }\n  }\n  P.bstart[P.nb] = at;",
                              "      at += cnt;\n    }\n    P.bstart[b] = at;\n  }\n  P.bstart[P.nb] = at;"),
    "par_drop_bucket_last_row": ("  if (m) {\n    P->out_keys[row] = q[m - 1].key;", "  if (m && 0) {\n    P->out_keys[row] = q[m - 1].key;"),
    "par_skip_last_bucket": ("  if (or_run(threads, P.nb, or_par_scan, &P)) goto done;",
                             "  if (or_run(threads, P.nb - 1, or_par_scan, &P)) goto done;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name, monkeypatch):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    tmp = tempfile.mkdtemp()
    try:
        path = os.path.join(tmp, "oracle.c")
        open(path, "w").write(src.replace(old, new))
        lib = os.path.join(tmp, "liboracle.so")
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-pthread", "-o", lib, path])
        import ctypes
        mut = ctypes.CDLL(lib)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        mut.oracle_groupby.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, u64, vp, vp]
        mut.oracle_groupby.restype = ctypes.c_int64
        mut.oracle_groupby_par.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, u64, vp, vp, u32, u32]
        mut.oracle_groupby_par.restype = ctypes.c_int64
        monkeypatch.setattr(oracle, "_lib", None)
        real_load = oracle._load

        def fake_load():
            real = real_load()
            class L:
                oracle_groupby = mut.oracle_groupby
                oracle_groupby_par = mut.oracle_groupby_par
                oracle_rows_for_keys = real.oracle_rows_for_keys
                oracle_totals = real.oracle_totals
            return L
        monkeypatch.setattr(oracle, "_load", fake_load)
        # a mutant of code both forms share must fail the single-threaded pin; one of the
        # parallel form's own code must fail the parallel pin
        form = oracle.groupby_par if name.startswith("par_") else oracle.groupby
        caught = False
        rng = np.random.default_rng(2024)
        for layout, gen, spec in (("R16", _rand_r16, SPEC_R16), ("R24", _rand_r24, SPEC_R24), ("MIX", _rand_mix, SPEC_MIX)):
            for _ in range(40):
                rec = gen(rng, int(rng.integers(1, 120)), _pool(rng, int(rng.integers(1, 20))))
                got = form(rec, spec, threads=3, bits=4) if form is oracle.groupby_par else form(rec, spec)
                if not _same(got, brute_force(rec, spec)):
                    caught = True
                    break
            if caught:
                break
        assert caught, f"mutant {name} survived the brute-force pin"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)

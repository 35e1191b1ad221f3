"""The C-ABI library builds, loads and exports every symbol include/aggx.h declares,
and its host-side validation rejects bad specs -- all without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "aggx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(agg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1311_0059_amd as P
    lib = P.load_library()
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert set(declared) == set(P.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_strerror_and_min_budget():
    import paper_1311_0059_amd as P
    lib = P.load_library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.agg_strerror(code)
    s = P.make_spec(16, [(0, "u64")], [("COUNT", 0, "i64")])
    assert 0 < P.min_budget(s) <= 16 << 20


@pytest.mark.parametrize("bad", [
    dict(record_bytes=15),
    dict(record_bytes=0),
    dict(keys=[(0, "u64"), (8, "u64")]),   # composite keys must be two u32 fields
    dict(keys=[(12, "u64")]),              # key past the record
    dict(keys=[(4, "u64")]),               # misaligned
    dict(aggs=[("SUM", 12, "i64")]),
    dict(aggs=[]),
    dict(aggs=[("COUNT", 0, "i64")] * 8, n_aggs=9),
    dict(load_pct=99),
    dict(fanout_bits=13),
])
def test_invalid_specs_rejected(bad):
    import paper_1311_0059_amd as P
    args = dict(record_bytes=16, keys=[(0, "u64")], aggs=[("COUNT", 0, "i64"), ("SUM", 8, "i64")])
    args.update(bad)
    n_aggs = args.pop("n_aggs", None)
    spec = P.make_spec(args.pop("record_bytes"), args.pop("keys"), args.pop("aggs"), **args)
    if n_aggs is not None:
        spec.n_aggs = n_aggs
    h = ctypes.c_void_p()
    rc = P.load_library().agg_create(ctypes.byref(spec), ctypes.byref(h))
    assert rc == -1 and not h.value


def test_budget_below_minimum_rejected():
    import paper_1311_0059_amd as P
    spec = P.make_spec(16, [(0, "u64")], [("COUNT", 0, "i64")], budget=4096)
    h = ctypes.c_void_p()
    assert P.load_library().agg_create(ctypes.byref(spec), ctypes.byref(h)) == -2


def test_null_arguments():
    import paper_1311_0059_amd as P
    lib = P.load_library()
    assert lib.agg_create(None, None) == -1
    assert lib.agg_consume(None, None, 0) == -1
    assert lib.agg_finish(None, None) == -1
    lib.agg_destroy(None)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C header gives its structs."""
    import ctypes
    import subprocess
    from paper_1311_0059_amd import _native as N
    pairs = {"agg_spec": N.Spec, "agg_result": N.Result, "agg_stats": N.Stats, "agg_instance": N.Instance,
             "agg_batch_stats": N.BatchStats, "agg_server_config": N.ServerConfig,
             "agg_request_info": N.RequestInfo, "agg_server_stats": N.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{ROOT}/include/aggx.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "in" if fname == "in_" else fname
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = pairs[cname]
        got = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(val), f"{cname}.{field}: ctypes {got} vs C {val}"

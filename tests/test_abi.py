"""CPU tests of the C-ABI library: it loads, exports every symbol include/wmh.h declares, and
its host-only logic (the bounds tables of Sec. 3.1 / Algorithm 4) is right.  No GPU needed."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1602_08393_amd import wmh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "wmh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wmh_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(wmh.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return wmh.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "wmh_hash" in names and "wmh_set_bounds" in names and "wmh_estimate" in names
    out = subprocess.run(["nm", "-D", "--defined-only", wmh.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (wmh_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)
    assert sorted(wmh.EXPORTED) == names


def test_opts_defaults(lib):
    o = wmh.WmhOpts()
    lib.wmh_opts_init(ctypes.byref(o))
    assert (o.mode, o.batch_rows, o.validate, o.use_graph, o.sync) == (0, 8192, 1, 1, 1)
    assert (o.rows_per_block, o.hashes_per_tile, o.stream_depth, o.waves_per_block) == (0, 0, 0, 0)
    assert o.values == 0
    assert o.coarse_bits == 0
    assert ctypes.sizeof(wmh.WmhOpts) == 4 * 17


def test_status_strings(lib):
    for code, name in wmh.STATUS.items():
        assert lib.wmh_status_string(code).decode() == name
    assert lib.wmh_status_string(-77).decode() == "WMH_E_UNKNOWN"


def test_null_context_is_rejected(lib):
    assert lib.wmh_set_bounds(None, None, 0) == -1
    assert lib.wmh_hash(None, None, None, None, 0, 0, 1, 0, None, None, None) == -1
    assert lib.wmh_last_error(None) == b""
    lib.wmh_destroy(None)


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = ctypes.c_void_p()
    assert lib.wmh_create(0, ctypes.byref(p)) != 0
    assert not p.value


def brute_bucket(prefix, D, q):
    """max{i < D : P[i] <= q} by linear scan."""
    best = 0
    for i in range(D):
        if int(prefix[i]) <= q:
            best = i
    return best


@pytest.mark.parametrize("seed", range(12))
def test_bounds_tables_against_brute_force(lib, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    D = int(rng.integers(1, 300))
    kind = seed % 4
    if kind == 0:
        m = rng.integers(0, 10, size=D)
    elif kind == 1:
        m = rng.integers(0, 2 ** 32, size=D)
    elif kind == 2:  # clustered tiny pieces between huge ones
        m = np.where(rng.random(D) < 0.9, rng.integers(0, 2, size=D), rng.integers(2 ** 30, 2 ** 32, size=D))
    else:
        m = np.ones(D)
    m = m.astype(np.uint32)
    if int(m.astype(np.uint64).sum()) == 0:
        m[0] = 1
    t = wmh.bounds_tables(m)
    P = np.concatenate([[0], np.cumsum(m.astype(np.uint64))]).astype(np.uint64)
    assert np.array_equal(t["prefix"], P)
    M = int(P[-1])
    target = 2
    while target < D:
        target *= 2
    target *= 2
    s = t["shift"]
    assert -(-M // (1 << s)) <= target
    assert s == 0 or -(-M // (1 << (s - 1))) > target
    assert t["n_buckets"] == -(-M // (1 << s))
    assert t["threshold"] == (1 << 64) % M
    for b in range(t["n_buckets"] + 1):
        assert int(t["bucket"][b]) == brute_bucket(P, D, b << s), b
    # every position's component lies in [T[b], T[b+1]]
    for p in rng.integers(0, M, size=200):
        c = int(np.searchsorted(P[:D], p, side="right")) - 1
        b = int(p) >> s
        assert t["bucket"][b] <= c <= t["bucket"][b + 1]


def test_bounds_tables_errors(lib):
    with pytest.raises(wmh.WMHError) as e:
        wmh.bounds_tables(np.zeros(5, dtype=np.uint32))
    assert e.value.name == "WMH_E_OVERFLOW"
    with pytest.raises(wmh.WMHError) as e:
        wmh.bounds_tables(np.zeros(0, dtype=np.uint32))
    assert e.value.name == "WMH_E_ARG"


def test_package_import_does_not_load_native_code():
    import sys
    import importlib
    import paper_1602_08393_amd
    importlib.reload(paper_1602_08393_amd)
    assert "oracle" not in paper_1602_08393_amd.__dict__
    src = open(os.path.join(ROOT, "paper_1602_08393_amd", "wmh.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for name in os.listdir(os.path.join(ROOT, "paper_1602_08393_amd", "csrc")):
        text = open(os.path.join(ROOT, "paper_1602_08393_amd", "csrc", name)).read()
        assert "oracle" not in text.lower(), name
    assert sys.modules.get("paper_1602_08393_amd") is not None


def test_host_pair_estimate(lib):
    rng = np.random.Generator(np.random.PCG64(3))
    for k in (1, 7, 500, 4099):
        a = rng.integers(0, 6, size=k).astype(np.uint16)
        b = rng.integers(0, 6, size=k).astype(np.uint16)
        count, jhat = wmh.estimate_pair(a, b)
        want = sum(1 for j in range(k) if int(a[j]) == int(b[j]))
        assert count == want and jhat == want / k
    z = np.zeros(9, dtype=np.uint16)
    assert wmh.estimate_pair(z, z) == (9, 1.0)  # two empty rows
    c = ctypes.c_uint32()
    assert lib.wmh_estimate_pair(z.ctypes.data, z.ctypes.data, 0, ctypes.byref(c), None) == -1
    assert lib.wmh_estimate_pair(None, z.ctypes.data, 9, ctypes.byref(c), None) == -1
    assert lib.wmh_estimate_pair(z.ctypes.data, z.ctypes.data, 9, None, None) == -1


@pytest.mark.parametrize("cname,py", [("wmh_opts", "WmhOpts"), ("wmh_server_config", "ServerConfig"),
                                      ("wmh_serving_stats", "ServingStats"),
                                      ("wmh_tune_result", "TuneResult")])
def test_structure_layouts_match_the_header(cname, py, tmp_path):
    """Every field of the binding's ctypes mirror sits at the offset, with the size, that a C
    compiler gives the header's struct (a field added on one side only shifts the rest)."""
    st = getattr(wmh, py)
    fields = [f[0] for f in st._fields_]
    lines = [f'printf("%zu\\n", sizeof({cname}));']
    for f in fields:
        lines.append(f'printf("%zu %zu\\n", offsetof({cname}, {f}), sizeof((({cname} *)0)->{f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"wmh.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    assert int(out[0]) == ctypes.sizeof(st)
    for f, line in zip(fields, out[1:]):
        off, size = map(int, line.split())
        assert (getattr(st, f).offset, getattr(st, f).size) == (off, size), f

"""CPU tests of the HIP library's host side (no GPU calls): the shared
library loads, exports every entry point include/lbm.h declares, and its
integer geometry (seeded electrodes, biofilm layer, link masks, link list,
percolation, growth pick) is byte-equal to the oracle's independent code."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1802_07525_amd as L
from paper_1802_07525_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = _header_functions()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares a signature for every header function
    assert set(names) <= set(L.exported_symbols())


def test_status_strings_and_version():
    lib = L.load()
    assert lib.lbm_status_str(0) == b"LBM_OK"
    assert lib.lbm_status_str(-4) == b"LBM_EDIVERGED"
    assert b"gfx950" in lib.lbm_version()


@pytest.mark.parametrize("seed", range(1, 9))
@pytest.mark.parametrize("overlap,fs", [(0, 0.3), (1, 0.55)])
def test_discs_byte_equal_to_oracle(seed, overlap, fs):
    st, a, fa = L.lbm_geom_discs(160, 80, 3, 6, fs, overlap, seed)
    so, b, fb = O.geom_discs(160, 80, 3, 6, fs, overlap, seed)
    assert st == 0 and so == "OK"
    assert np.array_equal(a, b) and fa == fb


@pytest.mark.parametrize("key", ["c1", "c5"])
def test_workload_masks_byte_equal(key):
    w = inputs.WORKLOADS[key]
    _, a, _ = L.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"], w["overlap"],
                               w["seed"])
    _, b, _ = O.geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"], w["overlap"],
                           w["seed"])
    a, b = L.lbm_biofilm_layer(a), O.biofilm_layer(b)
    assert np.array_equal(a, b)
    for which in (0, 1):
        assert np.array_equal(L.lbm_links(a, which), O.links(b, which))


@pytest.mark.parametrize("seed", [3, 4])
def test_fibres_and_3d_links_byte_equal(seed):
    st, a, fa = L.lbm_geom_fibres(48, 24, 20, 2, 4, 0.2, seed)
    so, b, fb = O.geom_fibres(48, 24, 20, 2, 4, 0.2, seed)
    assert st == 0 and np.array_equal(a, b) and fa == fb
    a, b = L.lbm_biofilm_layer(a), O.biofilm_layer(b)
    assert np.array_equal(a, b)
    for which in (0, 1):
        la, lb = L.lbm_links(a, which), O.links(b, which)
        assert la.dtype == lb.dtype and np.array_equal(la, lb)
    assert L.lbm_percolates(a) == O.percolates(b)


def test_link_list_is_ascending_set_bits():
    _, a, _ = L.lbm_geom_discs(64, 32, 2, 4, 0.3, 0, 7)
    a = L.lbm_biofilm_layer(a)
    for which, q in ((0, 9), (1, 5)):
        lst = L.lbm_link_list(a, which)
        bits = O.links(a, which).ravel()
        want = [(n, i) for n in range(a.size) for i in range(1, q) if (int(bits[n]) >> i) & 1]
        assert [tuple(r) for r in lst] == want


def test_percolation_and_growth_pick_match_oracle():
    rng = np.random.default_rng(5)
    for seed in range(1, 15):
        _, a, _ = L.lbm_geom_discs(64, 24, 2, 4, 0.25, 0, seed)
        a = L.lbm_biofilm_layer(a)
        assert L.lbm_percolates(a) == O.percolates(a)
        C = rng.random(a.size) - 0.05
        for xi in rng.random(5):
            assert L.lbm_growth_pick(a, C, xi) == O.growth_pick(a, C, xi)


def test_percolation_and_growth_pick_random_masks():
    rng = np.random.default_rng(9)
    for _ in range(40):
        a = (rng.random((10, 14)) < 0.42).astype(np.uint8) * rng.integers(1, 4, size=(10, 14)).astype(np.uint8)
        a[0] = 2
        a[-1] = 2
        assert L.lbm_percolates(a) == O.percolates(a)
        C = rng.random(a.size) - 0.1
        xi = float(rng.random())
        assert L.lbm_growth_pick(a, C, xi) == O.growth_pick(a, C, xi)


@pytest.mark.parametrize("shape", [(12, 17), (7, 9, 11), (5, 6, 40)])
def test_flow_domain_random_masks_match_oracle(shape):
    """The library searches over runs of FLUID nodes, the oracle node by
    node; random masks exercise every diagonal and edge link rule."""
    rng = np.random.default_rng(len(shape) * 100 + shape[-1])
    for frac in (0.25, 0.35, 0.45, 0.55):
        for _ in range(15):
            a = (rng.random(shape) < frac).astype(np.uint8) * rng.integers(1, 4, size=shape).astype(np.uint8)
            assert np.array_equal(L.lbm_flow_domain(a), O.flow_domain(a))
            assert L.lbm_percolates(a) == O.percolates(a)


def test_flow_domain_matches_oracle():
    for seed in range(1, 10):
        _, a, _ = L.lbm_geom_discs(96, 48, 2, 5, 0.35, 0, seed)
        a = L.lbm_biofilm_layer(a)
        assert np.array_equal(L.lbm_flow_domain(a), O.flow_domain(a))
    st, a, _ = L.lbm_geom_fibres(24, 12, 12, 1, 2, 0.35, 3)
    assert np.array_equal(L.lbm_flow_domain(a), O.flow_domain(a))


def test_splitmix64_matches_oracle():
    for seed in (0, 1, 1234567, 2 ** 63 + 11):
        assert np.array_equal(L.lbm_splitmix64(seed, 64), O.splitmix64(seed, 64))


def test_geometry_rejects_bad_arguments():
    st, _, _ = L.lbm_geom_discs(3, 2, 3, 6, 0.3, 0, 1)
    assert st == L.LBM_EINVAL
    st, _, _ = L.lbm_geom_discs(64, 32, 6, 3, 0.3, 0, 1)
    assert st == L.LBM_EINVAL
    # unreachable target with non-overlapping discs -> EINVAL after 10^6 attempts
    st, _, _ = L.lbm_geom_discs(16, 10, 5, 5, 0.9, 0, 1)
    assert st == L.LBM_EINVAL


def test_smoke_mask_percolates():
    """The smoke check's mask must be one the solver accepts."""
    import __graft_entry__ as G
    w = inputs.scaled(inputs.WORKLOADS["c1"], 96, 48, **G.SMOKE_MASK)
    st, cls, _ = L.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                    w["overlap"], w["seed"])
    assert st == 0
    assert L.lbm_percolates(L.lbm_biofilm_layer(cls))


def test_oracle_and_product_are_independent():
    """The oracle imports nothing of the product package and the product
    imports nothing of the oracle; the library's sources include nothing
    from oracle/ and the oracle's C includes nothing from the library."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1802_07525_amd")
    orc = os.path.join(root, "oracle")
    for d, banned in ((orc, r"paper_1802_07525_amd|_lbm"), (pkg, r"\boracle\b")):
        for dirpath, _, files in os.walk(d):
            for fn in files:
                if not fn.endswith((".py", ".c", ".h", ".cpp", ".hip")):
                    continue
                text = open(os.path.join(dirpath, fn)).read()
                for line in text.splitlines():
                    s = line.strip()
                    if s.startswith(("import ", "from ", "#include")):
                        assert not re.search(banned, s), (fn, s)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message (and
    before touching a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_counter_key_ignores_comments_and_trace_ranges():
    """The key that ties stored HBM counters to the kernels' code changes
    with code, not with comments or host-side roctx range statements."""
    import importlib
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    try:
        bench = importlib.import_module("bench")
    finally:
        sys.path.remove(root)
    base = "int f(int a)\n{\n    return a + 1;\n}\n"
    ranged = "int f(int a) // one\n{\n    Range rg(a ? \"x.y\" : \"x.z\");\n    /* two */ return a + 1;\n}\n"
    assert bench._code_only(base) == bench._code_only(ranged)
    assert bench._code_only(base) != bench._code_only(base.replace("+ 1", "+ 2"))
    assert bench._code_only(base) != bench._code_only(base.replace("return", "g(); return"))


def test_built_library_opens_roctx_ranges(tmp_path):
    """The built library's roctx ranges (LBM_ROCTX), through the C ABI on
    the CPU: a generated electrode is one balanced lbm.geometry range on a
    stub marker library (tests/sanitize/roctx_stub.c); a library that
    cannot be opened leaves the call's result unchanged."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    stub = str(tmp_path / "libroctx_stub.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-fPIC", "-shared",
                    os.path.join(root, "tests", "sanitize", "roctx_stub.c"), "-o", stub, "-lpthread"],
                   check=True)
    code = ("import sys, hashlib; sys.path.insert(0, %r); import paper_1802_07525_amd as lbm; "
            "st, cls, _ = lbm.lbm_geom_fibres(24, 12, 12, 1, 2, 0.2, 5); "
            "st2, cls2, _ = lbm.lbm_geom_discs(64, 32, 2, 4, 0.3, 0, 7); "
            "print(st, st2, hashlib.sha256(cls.tobytes() + cls2.tobytes()).hexdigest())" % root)
    runs = {}
    for name, val in (("off", None), ("stub", stub), ("missing", str(tmp_path / "missing.so"))):
        env = {k: v for k, v in os.environ.items() if k != "LBM_ROCTX"}
        env["ROCTX_STUB_OUT"] = str(tmp_path / ("%s.txt" % name))
        if val:
            env["LBM_ROCTX"] = val
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        runs[name] = r
    assert runs["off"].stdout == runs["stub"].stdout == runs["missing"].stdout
    assert runs["off"].stdout.startswith("0 0 ")
    assert "cannot open the roctx library" in runs["missing"].stderr
    assert not os.path.exists(str(tmp_path / "off.txt"))
    rec = dict(line.split(None, 1) for line in open(str(tmp_path / "stub.txt")))
    assert rec["pushes"].strip() == rec["pops"].strip() == "2"
    assert rec["bad_pops"].strip() == "0" and rec["unbalanced"].strip() == "0"
    assert rec["range"].strip() == "lbm.geometry 2"

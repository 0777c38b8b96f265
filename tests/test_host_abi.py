"""CPU tests of the C-ABI library: exported symbols, host small dense code
(real Schur form and reordering, the contraction of Algorithm 1) against LAPACK, and
argument validation that rejects bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

import paper_2508_05400_amd as P
from oracle.rks import which_key
from workloads import convdiff2d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)   # drop comments
            names |= set(re.findall(r"\b(rks_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    # and the binding knows all of them
    from paper_2508_05400_amd._binding import SIGNATURES
    assert set(declared) == set(SIGNATURES)


def test_strerror_and_defaults(lib):
    assert P.rks_strerror(0) == "ok"
    assert "invalid" in P.rks_strerror(-1)
    o = P.rks_opts_default()
    assert (o.zeta, o.max_restarts, o.lock, o.sketch_kind, o.precision) == (8, 300, 1, 1, 0)
    assert o.whiten_tol == 1e-12 and o.start_seed == 1


@pytest.mark.parametrize("seed", range(40))
def test_host_schur_matches_lapack(lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 90))
    A = rng.standard_normal((n, n))
    if seed % 3 == 1:
        A += 8 * np.triu(A, 1)            # strongly non-normal
    if seed % 3 == 2:
        A = np.diag(rng.standard_normal(n)) + 1e-6 * A
    T, Z = P.rks_host_schur(A)
    assert np.linalg.norm(Z @ T @ Z.T - A) <= 1e-13 * n * max(np.linalg.norm(A), 1)
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 1e-13 * n
    assert np.all(np.tril(T, -2) == 0)
    ev = np.sort_complex(np.linalg.eigvals(A))
    got = np.sort_complex(sla.eigvals(T))
    assert np.allclose(got, ev, atol=1e-9 * max(np.abs(ev).max(), 1))


@pytest.mark.parametrize("which", ["LM", "SM", "LR", "SR"])
@pytest.mark.parametrize("seed", range(10))
def test_host_order_selects_wanted(lib, which, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 70))
    A = rng.standard_normal((n, n)) + (3 * np.triu(rng.standard_normal((n, n)), 1) if seed % 2 else 0)
    T, Z = P.rks_host_schur(A)
    kw = max(1, n // 4)
    T2, Z2, p = P.rks_host_order(T, Z, which, kw)
    assert p in (kw, kw + 1)
    assert np.linalg.norm(Z2 @ T2 @ Z2.T - A) <= 1e-12 * n * np.linalg.norm(A)
    lead = sla.eigvals(T2[:p, :p])
    allv = np.linalg.eigvals(A)
    order = sorted(allv, key=lambda z: which_key(z, which), reverse=True)
    want = np.array(order[:p])
    assert np.allclose(np.sort_complex(lead), np.sort_complex(want), atol=1e-8 * np.abs(allv).max())
    # same invariant subspace as LAPACK's reordering (dtrsen) of the same set
    Tl, Zl = sla.schur(A, output="real")
    sel = np.zeros(n, dtype=np.int32)
    diag_ev = sla.eigvals(Tl)
    for z in want:
        sel[np.argmin(np.abs(diag_ev - z) + 1e9 * sel)] = 1
    Ts, Zs, *_ = sla.lapack.dtrsen(sel, Tl, Zl, job="N")
    s = np.linalg.svd(Zs[:, :p].T @ Z2[:, :p], compute_uv=False)
    assert s.min() > 1 - 1e-8


def test_create_rejects_bad_arguments(lib):
    A = convdiff2d(10)
    bad = [
        dict(k=0, m=10, d=20), dict(k=9, m=10, d=20), dict(k=3, m=10, d=10),   # k, m, d relation
        dict(k=3, m=10, d=200), dict(k=3, m=300, d=400),                      # d > n, m too large
    ]
    for b in bad:
        with pytest.raises(P.RksError) as ei:
            P.rks_create(A.row_ptr, A.col, A.val, A.n, b["k"], b["m"], b["d"], "LM", 1e-10)
        assert ei.value.code == -1
    with pytest.raises(P.RksError):
        P.rks_create(A.row_ptr, A.col, A.val, A.n, 3, 10, 20, "LM", 0.0)
    with pytest.raises(P.RksError):
        P.rks_create(A.row_ptr, A.col, A.val, A.n, 3, 10, 20, "LM", 1e-10, P.rks_opts_default(zeta=9))
    for lock in (-1, 3):  # 0 off, 1 leading blocks, 2 aggressive
        with pytest.raises(P.RksError) as ei:
            P.rks_create(A.row_ptr, A.col, A.val, A.n, 3, 10, 20, "LM", 1e-10, P.rks_opts_default(lock=lock))
        assert ei.value.code == -1
    for av in (-1, 2):  # 0 value-indexed when possible, 1 FP64 values
        with pytest.raises(P.RksError) as ei:
            P.rks_create(A.row_ptr, A.col, A.val, A.n, 3, 10, 20, "LM", 1e-10, P.rks_opts_default(a_values=av))
        assert ei.value.code == -1 and "a_values" in P.rks_last_error(None)
    # malformed CSR: decreasing row pointer, column out of range, unsorted row
    rp = A.row_ptr.copy(); rp[5] = rp[4] - 1
    with pytest.raises(P.RksError):
        P.rks_create(rp, A.col, A.val, A.n, 3, 10, 20, "LM", 1e-10)
    col = A.col.copy(); col[7] = A.n
    with pytest.raises(P.RksError):
        P.rks_create(A.row_ptr, col, A.val, A.n, 3, 10, 20, "LM", 1e-10)
    col = A.col.copy(); col[[10, 11]] = col[[11, 10]]
    with pytest.raises(P.RksError):
        P.rks_create(A.row_ptr, col, A.val, A.n, 3, 10, 20, "LM", 1e-10)
    val = A.val.copy(); val[3] = np.inf
    with pytest.raises(P.RksError) as ei:
        P.rks_create(A.row_ptr, A.col, val, A.n, 3, 10, 20, "LM", 1e-10)
    assert ei.value.code == -4


def test_product_path_has_no_oracle_dependency():
    """The library package must not import the oracle or fall back to the CPU."""
    pkg = os.path.join(ROOT, "paper_2508_05400_amd")
    for dp, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dp, fn)).read()
                assert "oracle" not in txt.lower(), fn


def test_learned_start_falls_back_to_random_without_weights(tmp_path):
    """No trained weights: the start is None, i.e. the solver's seeded random start."""
    from paper_2508_05400_amd.learned_start import start_for
    assert start_for(np.zeros((2, 64, 64)), 512, weights=str(tmp_path / "missing.npz")) is None


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of rks_csr, rks_opts and rks_stats have the C
    compiler's size and field offsets (a mismatch would corrupt memory)."""
    import shutil
    import subprocess
    from paper_2508_05400_amd import _binding as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"rks_csr": B.RksCsr, "rks_opts": B.RksOpts, "rks_stats": B.RksStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rks.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


def test_binding_enum_names_match_the_header(tmp_path):
    """The binding's string names for which, sketch kind, basis precision,
    SpMV layout, method and value storage map to the header's enum values (the precision
    names include the pair basis, "fp32+fx16")."""
    import shutil
    import subprocess
    from paper_2508_05400_amd import _binding as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    expect = {
        ("which", "LM"): "RKS_LM", ("which", "SM"): "RKS_SM", ("which", "LR"): "RKS_LR", ("which", "SR"): "RKS_SR",
        ("sketch", "gauss"): "RKS_SKETCH_GAUSS", ("sketch", "sparse"): "RKS_SKETCH_SPARSE",
        ("precision", "fp64"): "RKS_PREC_FP64", ("precision", "fp32"): "RKS_PREC_V32",
        ("precision", "bf16"): "RKS_PREC_VBF16", ("precision", "fp32+fx16"): "RKS_PREC_V32_FX16",
        ("layout", "auto"): "RKS_SPMV_AUTO", ("layout", "rows"): "RKS_SPMV_ROWS",
        ("layout", "column_blocks"): "RKS_SPMV_COLUMN_BLOCKS", ("layout", "sliced"): "RKS_SPMV_SLICED",
        ("method", "rks"): "RKS_METHOD_RKS", ("method", "ks_cgs2"): "RKS_METHOD_KS_CGS2",
        ("a_values", "auto"): "RKS_AVALUES_AUTO", ("a_values", "fp64"): "RKS_AVALUES_FP64",
    }
    tables = {"which": B.WHICH, "sketch": B.SKETCH, "precision": B.PRECISION, "layout": B.SPMV_LAYOUT,
              "method": B.METHOD, "a_values": B.A_VALUES}
    lines = ['#include <stdio.h>', '#include "rks.h"', "int main(void) {"]
    for (t, name), cname in expect.items():
        lines.append(f'  printf("{t} {name} %d\\n", (int){cname});')
    lines += ["  return 0;", "}"]
    src = tmp_path / "enums.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "enums"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        t, name, val = line.split()
        assert tables[t][name] == int(val), (t, name, tables[t][name], val)
        seen += 1
    assert seen == len(expect)
    # aliases map to values the header defines too
    for t, table in tables.items():
        assert set(table.values()) <= {tables[t][n] for (tt, n) in expect if tt == t}, t


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message before
    touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr

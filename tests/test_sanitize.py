"""The host small dense code (csrc/dense.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host only) and run on the dense steps of a
contraction: any out-of-bounds access, use after free, signed overflow or
other undefined operation aborts the run, and the harness checks the
identities the routines must satisfy (Schur backward error and orthonormal
vectors, the wanted eigenvalues leading after reordering, eigenvectors of the
quasi-triangular factor, Householder QR and the triangular inverse)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2508_05400_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_dense_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "dense_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{CSRC}", os.path.join(HERE, "sanitize", "dense_check.cpp"),
           os.path.join(CSRC, "dense.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
    assert run.stdout.strip().endswith("ok: 0 failures")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_panel_layout_under_asan_and_ubsan(tmp_path):
    """The column-blocked SpMV layout (csrc/panels.cpp) on matrices with empty
    rows, rows longer than a tile inside one column block (one beyond 16-bit
    offsets), fewer columns than blocks, a ragged last panel and the largest
    panel size: every nonzero lands once, every read the kernel makes stays
    in bounds, and a walk of the layout in the kernel's order reproduces the
    CSR product (64 u sum|terms|)."""
    exe = str(tmp_path / "panels_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{CSRC}", os.path.join(HERE, "sanitize", "panels_check.cpp"),
           os.path.join(CSRC, "panels.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
    assert run.stdout.strip().endswith("ok: 0 failures")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_slice_layout_under_asan_and_ubsan(tmp_path):
    """The sliced SpMV layout (slice_offsets, build_slices in csrc/panels.cpp)
    on matrices with empty rows, whole slices of empty rows, rows of up to 700
    nonzeros and ragged last slices: offsets padded to each slice's longest
    row, every nonzero once at its (slice, k, lane), every column a valid
    index of x, and the product in the kernel's order equal to the CSR
    product to the bit."""
    exe = str(tmp_path / "slices_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{CSRC}", os.path.join(HERE, "sanitize", "slices_check.cpp"),
           os.path.join(CSRC, "panels.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
    assert run.stdout.strip().endswith("ok: 0 failures")

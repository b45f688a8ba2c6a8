"""Host code under AddressSanitizer, on the CPU.

The oracle, built with the sanitizer, runs a small workload of every kind
(plans, Gaussians of strokes, fills and tangent-aligned strokes, compositing
and its adjoint, parameter gradients, the regularisers and the
distance-weighted loss); the C-ABI library, built with the sanitizer on its
host pass only, runs a C driver over its host entry points (sizes, tile
counts, workspace sizing, context error paths).  Either run fails on any
sanitizer report."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if p and os.path.exists(p) else None


ORACLE_RUN = r"""
import numpy as np, sys
sys.path.insert(0, %r)
import oracle
from paper_2606_31764_amd import synth
scenes = [synth._assemble(synth.strokes(11, n_curves=3, size=40, nk_range=(5, 8)), [[40, 44]], [[1.0, 1.0, 1.0]], 3),
          synth.config3(seed=12, n_paths=3, size=40),
          synth._assemble(synth.strokes(13, n_curves=2, size=40, nk_range=(5, 8), flags=synth.ANISO), [[40, 40]],
                          [[1.0, 1.0, 1.0]], 3)]
for b in scenes:
    p = dict(h=2.0, delta_c=2.0)
    pl, L, G = oracle.plan(b, p)
    g = oracle.gaussians(b, p)
    img = oracle.render(b, p)[0]
    loss, grads = oracle.loss_and_grad(b, np.full_like(img, 0.5), p)[:2]
    r = oracle.reg_loss(b, pl, p, bbox_weight=1.0, deriv_weight=0.1)
    u = oracle.udf_loss(b, pl, img, np.full_like(img, 0.4), 0.5, params=p)
    assert np.isfinite(img).all() and np.isfinite(loss)
print("oracle ok")
""" % ROOT


def test_oracle_under_asan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no libasan for this gcc")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fsanitize=address",
                           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "nsplat_oracle.cpp")])
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0", NSPLAT_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", ORACLE_RUN], env=env, capture_output=True, text=True, timeout=900)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "oracle ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


def test_library_host_code_under_asan(tmp_path):
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        pytest.skip("no ROCm clang")
    sys.path.insert(0, os.path.join(ROOT, "paper_2606_31764_amd"))
    import build as B
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    objs, procs = [], []
    for src in sorted(glob.glob(os.path.join(ROOT, "paper_2606_31764_amd", "csrc", "*.hip"))):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        # the sanitizer on the host pass only: device code is built as usual
        procs.append(subprocess.Popen(["hipcc", *flags, "-c", "-g", "-Xarch_host", "-fsanitize=address",
                                       "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(src), src, "-o", o],
                                      stderr=subprocess.DEVNULL))
        objs.append(o)
    assert all(p.wait(timeout=900) == 0 for p in procs)
    drv = str(tmp_path / "asan_host.o")
    subprocess.check_call([clang, "-c", "-g", "-x", "c", "-fsanitize=address", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "asan_host.c"), "-o", drv])
    exe = str(tmp_path / "asan_host")
    subprocess.check_call([clang, "-fsanitize=address", drv, *objs, "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-4000:])

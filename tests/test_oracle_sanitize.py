"""The oracle built with the address and undefined-behaviour sanitizers (host
only): on small matrices covering the edge cases (no arrow, no band, a dense
band, one tile, ragged tiles) it must run clean and give the same bits as the
ordinary build (both use -ffp-contract=off and no fast math, so the
optimisation level does not change the arithmetic)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2504_19171_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = [  # (nb, w, a, b)
    (150, 12, 5, 16),
    (97, 0, 3, 32),
    (64, 70, 0, 16),
    (40, 39, 7, 64),
    (200, 31, 0, 48),
    (130, 9, 18, 32),
]


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           os.path.join(ROOT, "oracle", "stiles_oracle.c"), os.path.join(HERE, "sanitize", "oracle_driver.c"),
           "-o", exe, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "sanitize" in res.stderr:
        pytest.skip("the sanitizer runtime is not available: " + res.stderr[-300:])
    assert res.returncode == 0, res.stderr
    return exe


@pytest.mark.parametrize("nb,w,a,b", CASES)
def test_sanitized_oracle_runs_clean_and_matches(sanitized_driver, oracle_mod, tmp_path, nb, w, a, b):
    M = inputs.arrowhead_spd(nb, w, a, seed=nb + 7 * w + a)
    wc = oracle_mod.clamp_w(nb, w)
    src = tmp_path / "in.bin"
    with open(src, "wb") as f:
        np.array([nb, wc, a, b], dtype=np.int64).tofile(f)
        np.ascontiguousarray(M.ab[: wc + 1], dtype=np.float64).tofile(f)
        if a:
            np.ascontiguousarray(M.P, dtype=np.float64).tofile(f)
            np.ascontiguousarray(M.C, dtype=np.float64).tofile(f)
    dst = tmp_path / "out.bin"
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([sanitized_driver, str(src), str(dst)], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr[-3000:]
    got = np.fromfile(dst, dtype=np.float64)
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, b)
    n = nb + a
    cols = [oracle_mod.sigma_column(f, j) for j in range(n)]
    ref = np.concatenate([np.array([f.logdet, float(f.info)]), f.Lr.ravel(), f.LP.ravel(), f.LC.ravel(),
                          S.Sb.ravel(), S.SP.ravel(), S.SC.ravel()] + cols)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref), f"max difference {np.max(np.abs(got - ref)):.3e}"

"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): a child process loads
the sanitized build of evp_oracle.c and runs its predictor and full steps over the cases the
parity tests use (periodic and channel with moving walls, the four closures, WENO5 and HOUC5,
artificial diffusion, AB2 and RK3).  Any out-of-bounds access or undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import oracle
from paper_1803_09563_amd import inputs

def state(shape, seed, walls):
    return inputs.random_state(shape, seed, walls=walls)

cases = 0
for walls in (False, True):
    nx, ny, nz = 12, 10 if walls else 8, 8
    g = oracle.Grid(nx, ny, nz, 2.0, 2.0 if walls else 1.5, 1.0, walls)
    for model in (oracle.OLDROYD_B, oracle.FENE_P, oracle.SARAMITO, oracle.NEO_HOOKEAN):
        for adv, kappa in ((oracle.WENO5, 0.0), (oracle.HOUC5, 0.0), (oracle.WENO5, 0.05)):
            r = oracle.Rheology(model, 1.0, 0.01, 0.02, 0.5, 0.002 if model == oracle.SARAMITO else 0.0,
                                50.0, adv, kappa)
            s = oracle.Solver(g, r, (oracle.FORCE_SIN_X_OF_Y, 0.1, 1.0),
                              (0.1, -0.1, 0.05, 0.0) if walls else (0.0, 0.0, 0.0, 0.0))
            u, v, w, B = state(g.shape, 7 + model, walls)
            s.write_fields(u, v, w, B)
            s.project()
            s.step(1e-3, 2)
            s.step(1e-3, 1, oracle.Solver.STOP_AFTER_PREDICTOR)
            s.step_rk3(1e-3, 1)
            assert all(np.isfinite(a).all() for a in (s.u, s.v, s.w, s.B, s.p))
            cases += 1
            s.health()
print("sanitized oracle cases:", cases)
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan)
    env = dict(os.environ)
    # the sanitizer runtime must come first; anything already preloaded stays after it
    env["LD_PRELOAD"] = asan + (" " + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env.update(EVP_ORACLE_LIB=so, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert "sanitized oracle cases: 24" in r.stdout, tail

"""The C ABI used from plain C: tests/c_abi_program.c (built by build() into
tests/_bin) lets the library allocate its own device arena and use the null
stream, advances a box 20 steps (10, a checkpoint into a new simulation, 10
more) and writes the state back. It must equal, bit for bit, the same run
through the Python binding (torch arena and stream) without the checkpoint."""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import random_state  # noqa: E402

pytestmark = pytest.mark.gpu
BIN = os.path.join(os.path.dirname(__file__), "_bin", "c_abi_program")
KEYS = ("x", "y", "ux", "uy", "qxx", "qxy", "rho", "ax", "ay")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def test_c_client_matches_python_binding(tmp_path):
    import paper_2108_08919_amd as P
    if not os.path.exists(BIN):
        pytest.fail("tests/_bin/c_abi_program is missing: run __graft_entry__.build()")
    side, steps = 32, 20
    s0 = random_state(side, 8, amp_u=2e-3)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.concatenate([np.asarray(s0[k], dtype=np.float64) for k in KEYS]).tofile(fin)
    r = subprocess.run([BIN, str(side), str(steps), str(fin), str(fout)], capture_output=True, text=True,
                       timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    raw = np.fromfile(fout, dtype=np.float64)
    n = side * side
    c_state = {k: raw[i * n:(i + 1) * n] for i, k in enumerate(KEYS)}
    c_diag = raw[9 * n:]
    p = wl.Params(L=float(side), zeta=0.02, K=0.02)
    sim = P.Sim([p], [n])
    sim.set_state(0, s0)
    sim.step(steps)
    sim.check()
    g = sim.get_state(0)
    d = sim.diagnostics(0)
    sim.close()
    for k in KEYS:
        assert np.array_equal(c_state[k], g[k]), k
    assert np.array_equal(c_diag, np.array([d[k] for k in ("px", "py", "ke", "F", "F_grad", "umax", "c0", "qmax")]))

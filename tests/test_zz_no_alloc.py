"""The entry point that allocates nothing, nem_defects_noalloc, against
nem_defects (which allocates its grid buffers on first use) through the C ABI:
identical defect counts on two calls in a row, the second with a smaller
input, on a fresh simulation and after other work; device memory unchanged by
the call; a grid beyond the static scratch refused with an explanation."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_08919_amd as P
    P.lib()
    yield


def say(*a):
    print(*a, flush=True)


def _sim(side, seed, steps):
    import paper_2108_08919_amd as P
    p = wl.Params(L=float(side), zeta=0.02, K=0.02)
    cfg = dict(n_side=side, params=p, kind="isotropic")
    sim = P.Sim([p], [side * side])
    sim.set_state(0, wl.state_for(cfg, seed))
    sim.step(steps)
    sim.check()
    return sim


def test_noalloc_defects_match_allocating_call():
    import torch
    import paper_2108_08919_amd as P
    say("noalloc: 512 box, M = 512 then 256")
    big = _sim(512, 0, 20)
    free = [torch.cuda.mem_get_info()[0]]
    a1 = big.defects_noalloc(0, 512)          # first call: no grid buffer exists yet
    free.append(torch.cuda.mem_get_info()[0])
    a2 = big.defects_noalloc(0, 256)          # second call, smaller grid
    free.append(torch.cuda.mem_get_info()[0])
    a3 = big.defects_noalloc(0, 512)
    free.append(torch.cuda.mem_get_info()[0])
    say("free device memory around the calls:", free)
    # The first launch of the deposit and winding kernels in a process may load
    # their code object (runtime, not the call); after it nothing changes.
    assert free[1] == free[2] == free[3]
    b1 = big.defects(0, 512)
    b2 = big.defects(0, 256)
    say("noalloc", a1, a2, "allocating", b1, b2)
    assert a1 == b1 and a2 == b2 and a3 == b1
    assert a1[0] > 1000 and a1[0] == a1[1]   # an isotropic start holds many +-1/2 pairs
    # after the allocating calls, in another simulation with a smaller box
    say("noalloc: 128 box, M = 128 then 64")
    small = _sim(128, 1, 10)
    c1 = small.defects_noalloc(0, 128)
    c2 = small.defects_noalloc(0, 64)
    assert c1 == small.defects(0, 128) and c2 == small.defects(0, 64)
    # and the big box again: the scratch keeps no state between calls
    assert big.defects_noalloc(0, 512) == b1
    # beyond the scratch: refused with an explanation, nothing run
    with pytest.raises(P.NemError) as ei:
        big.defects_noalloc(0, 1024)
    assert ei.value.code == P.NEM_E_INVAL and "512" in str(ei.value)
    big.close()
    small.close()

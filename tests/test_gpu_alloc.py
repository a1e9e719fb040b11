"""Device-memory hooks of pj_config (dev_alloc / dev_free), backed here by
torch's caching allocator: every device block the library takes comes from
the hook and goes back through it, joins give the same results as with the
library's own allocations, and an allocation failure injected at any point
of ingest or a join gives PJ_ERR_OUT_OF_MEMORY and leaks nothing."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


class CountingAlloc:
    def __init__(self, fail_after=None):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, n):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        p = self.torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        return p

    def free(self, p):
        self.torch.cuda.caching_allocator_delete(p)
        del self.live[p]


@pytest.fixture(scope="module")
def sets():
    return mg.config_multilod(seed=21, n_r=150, n_s=30, box=70.0)


def _run(pj, R, S, al, **cfg):
    import torch
    c = pj.Context(stream=torch.cuda.current_stream().cuda_stream, allocator=(al.alloc, al.free), **cfg)
    try:
        gR, gS = c.meshes(R), c.meshes(S)
        try:
            out = [c.join_within(gR, gS, tau) for tau in (0.0, 3.0)]
            out.append(c.join_knn(gR, gS, 2))
            return out
        finally:
            gR.close()
            gS.close()
    finally:
        c.close()


@pytest.mark.parametrize("cfg", [{}, dict(host_resident=True, mem_cap_bytes=64 << 20)])
def test_hooks_carry_every_allocation(sets, cfg):
    import paper_2604_19982_amd as pj
    R, S = sets
    al = CountingAlloc()
    got = _run(pj, R, S, al, **cfg)
    assert al.calls > 10 and not al.live, (al.calls, len(al.live))
    c = pj.Context(**cfg)
    gR, gS = c.meshes(R), c.meshes(S)
    want = [c.join_within(gR, gS, tau) for tau in (0.0, 3.0)] + [c.join_knn(gR, gS, 2)]
    for g, w in zip(got[:2], want[:2]):
        assert np.array_equal(g["r"], w["r"]) and np.array_equal(g["s"], w["s"])
    assert np.array_equal(got[2]["s"], want[2]["s"]) and np.array_equal(got[2]["dist"], want[2]["dist"])


def test_injected_allocation_failures_leak_nothing(sets):
    import paper_2604_19982_amd as pj
    R, S = sets
    total = CountingAlloc()
    _run(pj, R, S, total)
    n_calls = total.calls
    failed = 0
    for k in sorted(set(np.linspace(0, n_calls - 1, 12).astype(int).tolist())):
        al = CountingAlloc(fail_after=k)
        with pytest.raises(pj.PJError) as e:
            _run(pj, R, S, al)
        assert e.value.status == 2, (k, str(e.value))
        assert not al.live, (k, len(al.live))
        failed += 1
    print(f"{n_calls} allocations per run; {failed} injected failures, all OUT_OF_MEMORY without leaks", flush=True)
    # the device is still usable afterwards
    al = CountingAlloc()
    _run(pj, R, S, al)
    assert not al.live

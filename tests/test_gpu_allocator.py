"""Device memory and streams from the caller (the boundary's allocator
hook and stream pass-through): instances whose every buffer comes from
torch's caching allocator, on torch's stream, give the same results as
library-allocated ones; an allocator that fails at any point of creation or
of a run yields PAMC_ERR_OUT_OF_MEMORY with every block it handed out
returned (no leak), and the instance stays usable after a failed run."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pamc():
    from paper_2606_25203_amd import pamc as p
    return p


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Counting:
    """torch's caching allocator behind a counter; fail_at = k makes the
    k-th request (1-based) fail."""

    def __init__(self, pamc, torch, fail_at=0):
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_at = fail_at
        self.al = pamc.Allocator(self._alloc, self._free)

    def _alloc(self, n, stream):
        self.calls += 1
        if self.fail_at and self.calls == self.fail_at:
            return 0
        p = self.torch.cuda.caching_allocator_alloc(n, 0, stream)
        self.live[p] = n
        return p

    def _free(self, p, stream):
        assert p in self.live, "freed a block the allocator did not hand out"
        del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


AUG = dict(beta0=0.1, dbeta=0.05, augmented=1, z_rst=40, n_top=6, mis_trials=3, win_short=5, win_long=8, tau=4)


def run(pamc, inst, sched):
    res = inst.anneal(sched)
    return res, inst.state(), inst.best()[2]


def same(a, b):
    ra, sa, ba = a
    rb, sb, bb = b
    for f in ("best_cut", "steps_run", "n_cluster_moves", "n_reheats", "n_restarts"):
        assert getattr(ra, f) == getattr(rb, f), f
    assert ra.sum_lnq == rb.sum_lnq
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert np.array_equal(ba, bb)


@pytest.mark.parametrize("fields", ["pull", "push"])
def test_torch_memory_and_stream(pamc, torch, fields):
    g = synth.torus(24, 20, 3)
    sched = pamc.schedule(steps=60, sweeps=2, **AUG)
    say(f"case torch allocator + torch stream fields={fields}")
    ref = pamc.Instance.csr(g, replicas=128, seed=9, fields=fields)
    want = run(pamc, ref, sched)
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    stream = torch.cuda.Stream()  # default priority
    cnt = Counting(pamc, torch)
    inst = pamc.Instance.csr(g, replicas=128, seed=9, fields=fields, allocator=cnt.al, stream=stream.cuda_stream)
    info = inst.info()
    assert cnt.live and torch.cuda.memory_allocated() - base >= info.device_bytes
    got = run(pamc, inst, sched)
    same(got, want)
    # asynchronous primitives are ordered with torch work on the same stream
    inst.sweep(0.7, 3)
    with torch.cuda.stream(stream):
        marker = torch.ones(1, device="cuda")
    stream.synchronize()
    assert marker.item() == 1.0
    del marker
    inst.close()
    assert not cnt.live, f"{len(cnt.live)} blocks not returned"
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_allocation_failure_anywhere_in_creation(pamc, torch):
    g = synth.random_graph(301, 2500, 3)
    probe = Counting(pamc, torch)
    inst = pamc.Instance.csr(g, replicas=128, seed=2, allocator=probe.al)
    n_create = probe.calls
    inst.close()
    assert n_create > 5 and not probe.live
    say(f"case allocation failure at each of {n_create} creation requests")
    for k in range(1, n_create + 1):
        c = Counting(pamc, torch, fail_at=k)
        with pytest.raises(pamc.PamcError) as ex:
            pamc.Instance.csr(g, replicas=128, seed=2, allocator=c.al)
        assert ex.value.status == pamc.PAMC_ERR_OUT_OF_MEMORY, (k, ex.value)
        assert not c.live, f"request {k}: {len(c.live)} blocks leaked"


def hub_graph(n, m, seed):
    """A random graph plus one vertex joined to most others (its instances
    keep both field forms and switch within a run)."""
    rng = np.random.default_rng(seed)
    base = synth.random_graph(n, m, seed)
    us, vs = [], []
    for v in range(n):
        for e in range(base.row_ptr[v], base.row_ptr[v + 1]):
            if base.col[e] > v:
                us.append(v)
                vs.append(int(base.col[e]))
    for v in range(n):
        if rng.random() < 0.7:
            us.append(v)
            vs.append(n)
    return synth.csr_from_edges(n + 1, np.array(us), np.array(vs), np.ones(len(us), np.int32))


@pytest.mark.parametrize("graph", ["torus", "hub"])
def test_allocation_failure_in_a_run(pamc, torch, monkeypatch, graph):
    if graph == "hub":  # both field forms, switching at the step where beta reaches 0.8
        monkeypatch.setenv("PAMC_TILE", "0")
        g = hub_graph(200, 500, 3)
        sched = pamc.schedule(beta0=0.1, dbeta=0.05, steps=30, sweeps=2, augmented=1, z_rst=25, n_top=4,
                              mis_trials=2, tau=3)
    else:
        g = synth.torus(14, 10, 2)
        sched = pamc.schedule(steps=40, sweeps=2, **AUG)
    ref = pamc.Instance.csr(g, replicas=64, seed=4)
    want = run(pamc, ref, sched)
    ref.close()
    probe = Counting(pamc, torch)
    inst = pamc.Instance.csr(g, replicas=64, seed=4, allocator=probe.al)
    n0 = probe.calls
    inst.anneal(sched)
    n_run = probe.calls - n0  # the requests of the run itself (not of the snapshots after it)
    inst.close()
    assert n_run > 0
    say(f"case allocation failure at each of {n_run} run requests ({graph})")
    for k in range(1, n_run + 1):
        c = Counting(pamc, torch)
        inst = pamc.Instance.csr(g, replicas=64, seed=4, allocator=c.al)
        c.fail_at = c.calls + k
        with pytest.raises(pamc.PamcError) as ex:
            inst.anneal(sched)
        assert ex.value.status == pamc.PAMC_ERR_OUT_OF_MEMORY
        # still usable: a fresh population and the same run succeed
        inst.reset(4)
        same(run(pamc, inst, sched), want)
        inst.close()
        assert not c.live, f"request {k}: {len(c.live)} blocks leaked"


def test_server_with_torch_allocator(pamc, torch):
    sched = pamc.schedule(beta0=0.1, dbeta=0.1, steps=20, sweeps=2)
    reqs = [(synth.random_graph(100 + 50 * i, 400 + 100 * i, i), 30 + i) for i in range(5)]
    cnt = Counting(pamc, torch)
    say("case server on torch memory")
    srv = pamc.Server(1 << 30, 3, replicas=64, allocator=cnt.al)
    tickets = [srv.submit(g, s, sched) for g, s in reqs]
    srv.drain()
    for t, (g, s) in zip(tickets, reqs):
        inst = pamc.Instance.csr(g, replicas=64, seed=s)
        r = inst.anneal(sched)
        assert srv.poll(t).best_cut == r.best_cut
        inst.close()
    srv.close()
    assert not cnt.live

"""Allocation failures injected through the device-allocator hook of
ea_options: an allocator that refuses its k-th request, for every k that
ea_create makes, and for the staging buffers of ea_state / ea_set_state.
Each failure must come back as EA_ENOMEM with every buffer the call took
returned to the allocator, and a job running beside the failures must end in
exactly the state of the same job run without them (the chain of a job is a
fixed function of its inputs, Sec. 4.3.2 random stream; split calls give the
same chain)."""
import numpy as np
import pytest

from paper_1311_5582_amd import binding as B
from paper_1311_5582_amd import inputs

pytestmark = pytest.mark.gpu

L, R, N_T, SEED = 6, 3, 20, 77


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


class FailingAllocator(B.TorchAllocator):
    """Torch's caching allocator, except that request number fail_at
    (counting from 0) gets NULL."""

    def __init__(self, fail_at=None):
        super().__init__(0)
        self.calls = 0
        self.fail_at = fail_at

    def _alloc(self, nbytes, ctx):
        k = self.calls
        self.calls += 1
        if k == self.fail_at:
            return None
        return super()._alloc(nbytes, ctx)


def _job(allocator=None, **kw):
    J = inputs.couplings(L, R, SEED)
    betas = inputs.geometric_betas(N_T, 0.4, 2.0)
    return B.Sim(L, J, betas, SEED, allocator=allocator, **kw)


def _snapshot(sim):
    s, perm, t = sim.state()
    E, q = sim.observables()
    return s, perm, t, E, q, sim.swap_acceptance()


def _same(a, b):
    for x, y in zip(a, b):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y


@pytest.mark.parametrize("kw", [dict(), dict(layout="amsc4"), dict(rng="planes", split="always")])
def test_create_fails_cleanly_at_every_allocation(kw):
    counting = FailingAllocator()
    probe = _job(counting, **kw)
    n_allocs = counting.calls
    probe.close()
    assert n_allocs >= 10 and not counting.live
    twin = _job(**kw)
    per_step = 7
    for k in range(n_allocs):
        bad = FailingAllocator(k)
        with pytest.raises(B.EAError) as err:
            _job(bad, **kw)
        assert err.value.code == B.EA_ENOMEM, (k, str(err.value))
        assert bad.calls == k + 1, "allocation continued after a refusal"
        assert not bad.live, f"failure at allocation {k} leaked {len(bad.live)} buffers"
        twin.sweep(per_step, 1)
    ref = _job(**kw)
    ref.sweep(per_step * n_allocs, 1)
    _same(_snapshot(twin), _snapshot(ref))
    twin.close()
    ref.close()


def test_state_staging_failure_leaves_job_unchanged():
    alloc = FailingAllocator()
    job = _job(alloc)
    ref = _job()
    job.sweep(50, 1)
    good = job.state()

    alloc.fail_at = alloc.calls          # the staging buffer of the next readout
    with pytest.raises(B.EAError) as err:
        job.state()
    assert err.value.code == B.EA_ENOMEM

    spins, perm, t = good
    flipped = np.ascontiguousarray(-spins)
    alloc.fail_at = alloc.calls          # the staging buffer of the next upload
    with pytest.raises(B.EAError) as err:
        job.set_state(flipped, perm, t)
    assert err.value.code == B.EA_ENOMEM
    _same(job.state(), good)             # nothing of the refused upload arrived

    job.sweep(50, 1)
    ref.sweep(100, 1)
    _same(_snapshot(job), _snapshot(ref))
    live_before_close = len(alloc.live)
    job.close()
    assert live_before_close > 0 and not alloc.live
    ref.close()

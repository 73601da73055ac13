"""lecqmc_sweep_batch_static (the batched sweep that allocates no device
memory: descriptors staged in the library's fixed per-device array) against
lecqmc_sweep_batch on twin walkers: two calls in a row, the second with a
smaller batch, bit-identical states, weights and estimators; a batch above
the array's size and a repeated walker are refused."""
import numpy as np
import pytest

from paper_2601_08552_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    from paper_2601_08552_amd import lecqmc
    lecqmc.load()
    return lecqmc


def _cases():
    # uneven shapes: register tiles T = 1, 2, 4, the memory-inverse and the
    # delayed chain, FP64 and mixed precision
    return [
        (W.square_lattice(4), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=4, n_up=2, n_dn=2)),
        (W.square_lattice(8), dict(U=4.0, beta=1.0, dtau=0.1, n_stab=10, n_up=12, n_dn=12)),
        (W.square_lattice(6), dict(U=4.0, beta=0.6, dtau=0.1, n_stab=3, n_up=20, n_dn=17)),
        (W.flat_band_chain(4), dict(U=2.0, beta=1.0, dtau=0.05, n_stab=6, n_up=2, n_dn=2, precision=1)),
        (W.periodic_chain(40), dict(U=2.0, beta=0.4, dtau=0.1, n_stab=2, n_up=34, n_dn=5)),
        (W.square_lattice(6), dict(U=3.0, beta=0.8, dtau=0.1, n_stab=4, n_up=5, n_dn=4)),
    ]


def _twins(lq, ctx):
    a, b = [], []
    for t, (lat, kw) in enumerate(_cases()):
        par = W.Params(seed=60 + t, walker_id=t, **kw)
        a.append(lq.Walker(ctx, lat, par))
        b.append(lq.Walker(ctx, lat, par))
    return a, b


def _assert_same(a, b):
    for wa, wb in zip(a, b):
        for x, y in zip(wa.state(), wb.state()):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert wa.tracked_weight() == wb.tracked_weight()
        assert np.array_equal(wa.measure(), wb.measure())
        sa, sb = wa.stats(), wb.stats()
        for k in ("flip_accepts", "swap_accepts", "sweeps"):
            assert sa[k] == sb[k], k


def test_static_batch_equals_allocating_batch(lq):
    ctx = lq.Context(0)
    alloc, static = _twins(lq, ctx)
    print("call 1: six walkers, two measured sweeps", flush=True)
    lq.sweep_batch(alloc, 2, measure=True)
    lq.sweep_batch_static(static, 2, measure=True)
    _assert_same(alloc, static)
    print("call 2: three walkers, one sweep", flush=True)
    lq.sweep_batch(alloc[:3], 1)
    lq.sweep_batch_static(static[:3], 1)
    _assert_same(alloc, static)
    ctx.close()


def test_static_batch_refusals(lq):
    ctx = lq.Context(0)
    lat, par = W.config_small(seed=2)
    w = lq.Walker(ctx, lat, par)
    before = w.state()
    with pytest.raises(lq.LecqmcError) as e:
        lq.sweep_batch_static([w, w], 1)
    assert e.value.code == lq.EINVAL
    with pytest.raises(lq.LecqmcError) as e:
        lq.sweep_batch_static([w] * (lq.STATIC_MAX_WALKERS + 1), 1)
    assert e.value.code == lq.EINVAL and "at most" in str(e.value)
    for x, y in zip(w.state(), before):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    ctx.close()

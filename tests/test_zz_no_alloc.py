"""aqt_run_noalloc, the entry point for callers that cannot allocate: the same outputs
as aqt_run bit for bit (same kernels, same fixed-order reduction), on calls in a row
that reuse the device buffer (a smaller run after a larger one, another context on the
same device), and its limits."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("pgs_sum", "pgs_sumsq", "jump_totals", "jump_count", "net_gs", "net_hist", "jumps", "final_state")


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def _outs(eng, K, cap):
    return eng.alloc_outputs(K, cap, final_state=True)


def _same(a, b):
    import torch
    for k in FIELDS:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
def test_noalloc_equals_run_on_consecutive_calls(prec):
    """256 levels: reference runs through aqt_run, then two no-allocation runs in a row,
    the second smaller (its per-tile sums overwrite the start of the first's)."""
    inst = W.pm1_all_to_all(8, 13, t_f=1.0e4, n_grid=200)
    eng = _engine(inst)
    cap = 96
    sizes = ((1003, 5), (77, 6))
    refs = []
    for K, seed in sizes:
        o = _outs(eng, K, cap)
        eng.run_into(o, K, prec, seed=seed, record_capacity=cap)
        refs.append(o)
    got = []
    for K, seed in sizes:
        o = _outs(eng, K, cap)
        eng.run_noalloc_into(o, K, prec, seed=seed, record_capacity=cap)
        got.append(o)
    eng.stream.synchronize()
    assert eng.run_status() == 0
    for r, g in zip(refs, got):
        _same(r, g)
    assert int(refs[0]["jump_totals"].sum()) > 1003


def test_noalloc_shared_buffer_across_contexts():
    """Two contexts on one device share the buffer: alternating calls of a 16-level and a
    256-level instance each reproduce their aqt_run outputs."""
    small = W.config_small()
    big = W.pm1_all_to_all(8, 13, t_f=1.0e4, n_grid=200)
    e1, e2 = _engine(small), _engine(big)
    cap = 96
    cases = [(e1, 1000, 3), (e2, 520, 4), (e1, 9, 5)]
    refs = []
    for eng, K, seed in cases:
        o = _outs(eng, K, cap)
        eng.run_into(o, K, "fp32", seed=seed, record_capacity=cap)
        refs.append(o)
    got = []
    for eng, K, seed in cases:
        o = _outs(eng, K, cap)
        eng.run_noalloc_into(o, K, "fp32", seed=seed, record_capacity=cap)
        got.append(o)
    for eng in (e1, e2):
        eng.stream.synchronize()
    for r, g in zip(refs, got):
        _same(r, g)


def test_noalloc_limits():
    """No resident operands for the precision -> AQT_ESTATE; per-tile sums beyond the
    buffer -> AQT_EINVAL; nothing is enqueued and the context stays usable."""
    from paper_1710_03431_amd.binding import AQT_EINVAL, AQT_ESTATE, AqtError
    inst = W.pm1_all_to_all(8, 13, t_f=1.0e4, n_grid=200)
    eng = _engine(inst)
    o = _outs(eng, 64, 0)
    with pytest.raises(AqtError) as e:
        eng.run_noalloc_into(o, 64, "fp64", seed=1)
    assert e.value.status == AQT_ESTATE
    eng.run_into(o, 64, "fp64", seed=1)
    K = 200_000    # tile 8: 25000 tiles x 200 points x 16 bytes = 80 MB > 64 MiB
    big = eng.alloc_outputs(K, 0, per_trajectory=False)
    with pytest.raises(AqtError) as e:
        eng.run_noalloc_into(big, K, "fp64", seed=1, tile=8)
    assert e.value.status == AQT_EINVAL
    o2 = _outs(eng, 64, 0)
    eng.run_noalloc_into(o2, 64, "fp64", seed=1)
    eng.stream.synchronize()
    np.testing.assert_array_equal(o2["pgs_sum"].cpu().numpy(), o["pgs_sum"].cpu().numpy())

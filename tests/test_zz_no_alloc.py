"""lbp_run_bp_until_noalloc (workspace in the library's fixed device array,
no device allocation) against lbp_run_bp_until on the same graphs: the
iterations run, the residual, the messages, beliefs and MAP are bitwise equal
(both run the same kernels).  Two calls in a row on the fixed array, the
second on a smaller graph, so stale contents of the first must not leak into
the second; a graph whose workspace exceeds the array is refused."""
import numpy as np
import pytest

from paper_2202_04110_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compare(lbp, ctx, spec, max_iters, d, T, tol, every, fused=False):
    ref = lbp.Graph(ctx, spec)
    g = lbp.Graph(ctx, spec)
    if fused:
        ref.use_fused(True)
        g.use_fused(True)
    want = ref.run_bp_until(max_iters, d, T, tol, check_every=every)
    got = g.run_bp_until_noalloc(max_iters, d, T, tol, check_every=every)
    print("%s: run_bp_until %s, noalloc %s" % (spec.name, want, got))
    assert got == want
    np.testing.assert_array_equal(g.get_messages(), ref.get_messages())
    np.testing.assert_array_equal(g.get_beliefs(), ref.get_beliefs())
    np.testing.assert_array_equal(g.decode_map(), ref.decode_map())
    g.free()
    ref.free()
    return got


def test_noalloc_matches_run_bp_until(gpu_lib):
    lbp = gpu_lib
    ctx = lbp.Context(0)
    # first call: a large graph (about 13 MB of the 64 MB array), fused
    # iterations between checks, stops early
    done, r = _compare(lbp, ctx, W.potts_grid(400, 5, 2), 300, 0.5, 1.0, 1e-3, 5, fused=True)
    assert done < 300 and r < 1e-3
    # second call: a smaller graph with logical factors, max-product, every
    # iteration checked, runs to its cap
    spec = W.deconv(seed=4, K=2, tw=4, sd=10, img=12)
    done, _ = _compare(lbp, ctx, spec, 40, 0.5, 0.0, 0.0, 1)
    assert done == 40
    # the same call again after the large one, and a cap below check_every
    _compare(lbp, ctx, W.potts_grid(24, 4, 31), 300, 0.5, 1.0, 1e-3, 7)
    _compare(lbp, ctx, W.ising_grid(9, 33), 3, 0.5, 0.0, 1e-3, 10)
    ctx.close()


def test_noalloc_refuses_graphs_beyond_the_array(gpu_lib):
    lbp = gpu_lib
    ctx = lbp.Context(0)
    g = lbp.Graph(ctx, W.potts_grid(1024, 5, 2))  # about 84 MB of message panels
    before = g.get_messages()
    with pytest.raises(lbp.LBPError) as ei:
        g.run_bp_until_noalloc(10, 0.5, 1.0, 1e-3)
    assert ei.value.code == lbp.LBP_E_UNSUPPORTED
    np.testing.assert_array_equal(g.get_messages(), before)  # nothing ran
    for bad in ((10, 0.5, 1.0, -1.0, 1), (10, 0.5, 1.0, 1e-3, 0), (-1, 0.5, 1.0, 1e-3, 1)):
        with pytest.raises(lbp.LBPError) as ei:
            g.run_bp_until_noalloc(*bad[:4], check_every=bad[4])
        assert ei.value.code == lbp.LBP_E_INVALID
    g.free()
    ctx.close()

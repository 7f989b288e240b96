"""The library's streaming bandwidth probes (lbp_bandwidth_probe): each kind
moves exactly the data it documents, reports a positive time below what any
HBM part allows, and malformed arguments are refused before a launch."""
import pytest

pytestmark = pytest.mark.gpu

N_BYTES = 64 << 20


def test_bandwidth_probes_move_the_documented_data(gpu_lib):
    import torch
    lbp = gpu_lib
    ctx = lbp.Context(0)
    try:
        nf = N_BYTES // 4
        a = torch.zeros(nf, dtype=torch.float32, device="cuda")
        b = torch.full((nf,), 7.0, dtype=torch.float32, device="cuda")

        def rate(ms, moved):
            gbps = moved / (ms * 1e-3) / 1e9
            assert 0.0 < gbps < 20000.0, gbps
            return gbps

        # read: src all zeros, so the sink is left as it was
        ms = ctx.bandwidth_probe(0, a, b, N_BYTES, 1024, reps=3)
        rate(ms, N_BYTES)
        torch.cuda.synchronize()
        assert float(b[0]) == 7.0

        # copy: small integers, so every value is exact
        a.copy_(torch.arange(nf, device="cuda", dtype=torch.int64).remainder(1000).to(torch.float32))
        ms = ctx.bandwidth_probe(1, a, b, N_BYTES, 1024, reps=3)
        rate(ms, 2 * N_BYTES)
        torch.cuda.synchronize()
        assert torch.equal(a, b)

        # write: zeros over the whole destination, nothing past it
        ms = ctx.bandwidth_probe(2, None, b[: nf - 4], N_BYTES - 16, 1024, reps=3)
        rate(ms, N_BYTES - 16)
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(b[: nf - 4])) == 0
        assert torch.equal(b[nf - 4:], a[nf - 4:])

        # five reads per write: dst float4 i = sum over k of src float4 i + k*m
        nb = (N_BYTES // 80) * 80
        m4 = nb // 80
        b.fill_(-1.0)
        ms = ctx.bandwidth_probe(3, a, b, nb, 1024, reps=3)
        rate(ms, nb + nb // 5)
        torch.cuda.synchronize()
        want = a[: nb // 4].view(5, m4 * 4).sum(0)
        assert torch.equal(b[: m4 * 4], want)
        assert bool((b[m4 * 4:] == -1.0).all())

        for kind, nbytes, blocks in ((4, N_BYTES, 64), (-1, N_BYTES, 64), (0, 0, 64), (0, 24, 64),
                                     (3, 96, 64), (1, N_BYTES, 0)):
            with pytest.raises(lbp.LBPError) as ei:
                ctx.bandwidth_probe(kind, a, b, nbytes, blocks, reps=1)
            assert ei.value.code == lbp.LBP_E_INVALID
        with pytest.raises(lbp.LBPError) as ei:
            ctx.bandwidth_probe(1, None, b, N_BYTES, 64, reps=1)  # a copy needs a source
        assert ei.value.code == lbp.LBP_E_INVALID
        with pytest.raises(lbp.LBPError) as ei:
            ctx.bandwidth_probe(1, a[1:], b, 1024, 64, reps=1)  # 4-byte aligned only
        assert ei.value.code == lbp.LBP_E_INVALID
    finally:
        ctx.close()

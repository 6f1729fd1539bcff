"""The measured-ceiling probes behind the roofline figures: lsq_read_bandwidth and lsq_copy_bandwidth run on
the device, the copy leaves dst equal to src, and the argument checks reject what the header says."""
import pytest

pytestmark = pytest.mark.gpu


def test_copy_and_read_ceilings():
    import torch

    from paper_1911_02675_amd import lsq
    ctx = lsq.Context()
    try:
        src = torch.randn(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.zeros_like(src)
        g = ctx.copy_bandwidth(src, dst, reps=2)
        torch.cuda.synchronize()
        print("copy ceiling", g, "GB/s", flush=True)
        assert torch.equal(src, dst)
        r = ctx.read_bandwidth(src, reps=2)
        print("read ceiling", r, "GB/s", flush=True)
        # both are rates of real transfers: positive and below the 8 TB/s HBM peak by construction of the
        # kernels (no caching trick can serve 1 GiB per repetition from the 4 MB L2s or the 256 MB memory-side cache)
        assert 100.0 < g < 8000.0 and 100.0 < r < 8000.0
        with pytest.raises(lsq.LsqError) as e:
            ctx.copy_bandwidth(src, src, reps=1)  # overlapping
        assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
        with pytest.raises(lsq.LsqError) as e:
            ctx.copy_bandwidth(src[1:], dst[1:], reps=1)  # misaligned
        assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
        with pytest.raises(lsq.LsqError) as e:
            ctx.copy_bandwidth(src, dst, reps=0)
        assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    finally:
        ctx.close()

"""dpg_retrieve_noalloc (the retrieval whose workspace is the library's static
device array) against dpg_retrieve with caller workspace, through the C ABI:
two calls in a row, the second smaller, for DPG and direct retrieval; a shape
whose workspace exceeds the array is refused and leaves dst untouched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_cs_0308004_amd import dpg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SCRATCH_BYTES = 64 << 20  # DPG_NOALLOC_SCRATCH_BYTES


def noalloc(ctx, src, rids, dst, algo, stream):
    return dpg.lib().dpg_retrieve_noalloc(ctx.handle, src.data_ptr(), src.shape[0], src.shape[1],
                                          rids.data_ptr(), rids.numel(), dst.data_ptr(), algo, 0,
                                          ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_matches_retrieve_two_calls():
    ctx = dpg.Context(0)
    stream = torch.cuda.current_stream()
    try:
        for algo in (dpg.ALGO_DPG, dpg.ALGO_DIRECT):
            # the second call is smaller than the first and finds the first
            # call's bytes in the array
            for n, m, rec in ((300007, 500000, 100), (5001, 7003, 36)):
                assert ctx.retrieve_workspace_bytes(n, rec, m, algo) <= SCRATCH_BYTES
                src = torch.from_numpy(synth.record_bytes(n, rec, seed=n)).to(DEV)
                rids = torch.from_numpy(synth.rids_uniform(n, m, seed=m)).to(DEV)
                want = ctx.retrieve(src, rids, algo=algo)
                dst = torch.full((m, rec), 7, dtype=torch.uint8, device=DEV)
                assert noalloc(ctx, src, rids, dst, algo, stream) == dpg.OK
                torch.cuda.synchronize()
                assert torch.equal(dst, want), f"algo {algo}, {m} rids of {rec} B"
        # DPG over 2^21 rids of 100 B (an output larger than the cache the
        # two-phase form writes through, so INTERNAL is in the workspace)
        # needs more than the array holds
        n = m = 1 << 21
        assert ctx.retrieve_workspace_bytes(n, 100, m, dpg.ALGO_DPG) > SCRATCH_BYTES
        src = torch.from_numpy(synth.record_bytes(n, 100, seed=3)).to(DEV)
        rids = torch.from_numpy(synth.rids_permutation(n, seed=3)).to(DEV)
        dst = torch.full((m, 100), 7, dtype=torch.uint8, device=DEV)
        assert noalloc(ctx, src, rids, dst, dpg.ALGO_DPG, stream) == dpg.ERR_WORKSPACE_TOO_SMALL
        torch.cuda.synchronize()
        assert bool((dst == 7).all())
        # direct retrieval of the same shape fits (256 bytes of workspace)
        assert noalloc(ctx, src, rids, dst, dpg.ALGO_DIRECT, stream) == dpg.OK
        torch.cuda.synchronize()
        assert np.array_equal(dst[::997].cpu().numpy(), src[rids[::997].long()].cpu().numpy())
    finally:
        ctx.close()

"""The autotuner: it times the candidate plans, records the fastest, AUTO then
follows the table, the table survives a save/load round trip, and every
candidate it ran left a correct result."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_cs_0308004_amd import dpg, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_autotune_records_and_auto_follows(tmp_path):
    with dpg.Context(0) as ctx:
        n, rec = 300000, 16
        src = synth.record_bytes(n, rec, seed=5)
        rids = synth.rids_permutation(n, seed=5)
        want = oracle.retrieve(src, rids)
        s_t, r_t = torch.from_numpy(src).to(DEV), torch.from_numpy(rids).to(DEV)
        assert ctx.tune_count() == 0
        best, ms = ctx.autotune_retrieve(s_t, r_t, reps=2)
        assert ms > 0 and ctx.tune_count() == 1
        assert best.algo in (dpg.ALGO_DIRECT, dpg.ALGO_DPG)
        auto = ctx.plan_retrieve(n, rec, n, dpg.ALGO_AUTO)
        assert auto.algo == best.algo
        if best.algo == dpg.ALGO_DPG:
            assert auto.log2_run == best.log2_run and auto.probe == best.probe
        out = ctx.retrieve(s_t, r_t, algo=dpg.ALGO_AUTO)
        assert np.array_equal(out.cpu().numpy(), want)
        # best DPG configuration only
        bd, _ = ctx.autotune_retrieve(s_t, r_t, reps=1, dpg_only=True)
        assert bd.algo == dpg.ALGO_DPG
        # the reported plan is the one AUTO now uses, field by field
        auto = ctx.plan_retrieve(n, rec, n, dpg.ALGO_AUTO)
        for field, _ in dpg.Plan._fields_:
            assert getattr(auto, field) == getattr(bd, field), field
        assert bd.gather in (dpg.GATHER_CACHED, dpg.GATHER_LDS, dpg.GATHER_NONE)
        path = os.path.join(tmp_path, "tune.txt")
        ctx.tune_save(path)
        ctx.tune_clear()
        assert ctx.tune_count() == 0
        ctx.tune_load(path)
        assert ctx.tune_count() == 1
        assert ctx.plan_retrieve(n, rec, n, dpg.ALGO_AUTO).algo == bd.algo
        with open(path, "a") as f:
            f.write("16 19 19 7 0 0 0 1.0\n")
        with pytest.raises(dpg.DPGError):
            ctx.tune_load(path)

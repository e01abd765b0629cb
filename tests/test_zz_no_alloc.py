"""The allocation-free MV entry point (mrv_mv_device_noalloc) against
mrv_mv_device on the same device-resident inputs: identical booleans on two
calls in a row, the second with a smaller input, and no device memory taken
from the context's arena by either call."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2604_23960_amd import mrv
from paper_2604_23960_amd import workloads as W

pytestmark = pytest.mark.gpu

FLAG_SETS = [mrv.CHECK_ENV | mrv.EXHAUSTIVE, mrv.CHECK_ENV, 0]


def say(*a):
    print("[case]", *a, flush=True)


def test_noalloc_matches_device_entry_point():
    import torch
    torch.cuda.set_device(0)
    w = W.arms_workload(3000)
    small = w.paths.subset(np.arange(2300, 3000))
    arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    ctx = mrv.Context(0, device_arena=arena)
    try:
        team, env = ctx.load_team(w.team), ctx.load_env(w.env)
        inputs = [mrv.DevicePaths(w.paths), mrv.DevicePaths(small)]
        before = ctx.memory_stats()
        got = {}
        # two calls in a row per flag set, the second smaller, queued back to back
        for flags in FLAG_SETS:
            for k, dp in enumerate(inputs):
                say("noalloc", flags, dp.n_queries)
                out = torch.full((dp.n_queries,), 7, dtype=torch.uint8, device="cuda")
                ctx.mv_device_noalloc(team, env, dp, flags, out.data_ptr())
                got[flags, k] = out
        ctx.sync()
        after = ctx.memory_stats()
        assert after["used"] == before["used"] and after["peak"] == before["peak"], (before, after)
        for flags in FLAG_SETS:
            for k, dp in enumerate(inputs):
                say("mv_device", flags, dp.n_queries)
                ref = torch.full((dp.n_queries,), 9, dtype=torch.uint8, device="cuda")
                ctx.mv_device(team, env, dp, flags, ref.data_ptr())
                ctx.sync()
                a, b = got[flags, k].cpu().numpy(), ref.cpu().numpy()
                assert set(np.unique(b)) <= {0, 1}
                assert np.array_equal(a, b), (flags, k, np.flatnonzero(a != b)[:10])
        # the smaller call also against the FP64 oracle
        ot, oe, op = oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(small)
        assert np.array_equal(got[mrv.CHECK_ENV, 1].cpu().numpy(), oracle.mv(ot, oe, op))
        assert np.array_equal(got[0, 1].cpu().numpy(), oracle.mv(ot, oe, op, check_env=False))
    finally:
        ctx.close()


def test_noalloc_rejects_oversized_calls():
    import torch
    torch.cuda.set_device(0)
    w = W.arms_workload(16)
    ctx = mrv.Context(0)
    try:
        team, env = ctx.load_team(w.team), ctx.load_env(w.env)
        dp = mrv.DevicePaths(w.paths)
        out = torch.full((16,), 7, dtype=torch.uint8, device="cuda")
        # rejected on the host before any device array is read
        desc = mrv.PathsDesc(mrv.NOALLOC_MAX_QUERIES + 1, dp.desc.dof_stride, dp.desc.wp_begin, dp.desc.wp_t,
                             dp.desc.wp_q, dp.desc.n_wp)
        st = mrv.lib().mrv_mv_device_noalloc(ctx.h, team, env, C.byref(desc), mrv.CHECK_ENV, out.data_ptr())
        assert st == mrv.MRV_E_INVALID
        assert "MRV_NOALLOC_MAX_QUERIES" in mrv.last_error()
        st = mrv.lib().mrv_mv_device_noalloc(ctx.h, team + 1000, env, C.byref(dp.desc), 0, out.data_ptr())
        assert st == mrv.MRV_E_HANDLE
        ctx.sync()
        assert np.all(out.cpu().numpy() == 7)
        # and a valid call afterwards still answers
        ctx.mv_device_noalloc(team, env, dp, mrv.CHECK_ENV, out.data_ptr())
        ctx.sync()
        assert np.array_equal(out.cpu().numpy(),
                              oracle.mv(oracle.Team(w.team), oracle.Env(w.env), oracle.Paths(w.paths)))
    finally:
        ctx.close()

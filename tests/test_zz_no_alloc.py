"""GPU test of gnm_classify_flag_static, the variant of gnm_classify_flag that
allocates nothing and keeps its partial tables in the library's static
device scratch.  Through the C ABI, its tables and flags must equal
gnm_classify_flag's with a caller workspace, bit for bit, on two calls in a
row, the second with a smaller input (so stale scratch contents of the first
call must not leak into it); the oracle is checked too.  A launch whose
partial tables would pass the scratch, and a caller workspace, are rejected
before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from tests._gpu import DEV, diff, offsets_to_device, to_device

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(reg, rec, off, threshold=1_000_000, min_bulk=0, grid_blocks=0):
    """(static tables, static flags, workspace tables, workspace flags) as numpy."""
    import torch
    nw = 1 if off is None else len(off) - 1
    d = to_device(rec)
    doff = None if off is None else offsets_to_device(off)
    acc_s = torch.full((nw, reg.rows, 8), 0x5A5A, dtype=torch.int64, device=DEV)
    fl_s = torch.full((nw * reg.n_sites,), 0xA5, dtype=torch.uint8, device=DEV)
    gnm.classify_flag_static(reg, d, acc_s, fl_s, threshold, min_bulk, window_offsets=doff, n_windows=nw,
                             n=rec.n, grid_blocks=grid_blocks)
    acc_w = torch.full((nw, reg.rows, 8), 0x3C3C, dtype=torch.int64, device=DEV)
    fl_w = torch.full((nw * reg.n_sites,), 0x5A, dtype=torch.uint8, device=DEV)
    gnm.classify_flag(reg, d, acc_w, fl_w, threshold, min_bulk, window_offsets=doff, n_windows=nw, n=rec.n,
                      grid_blocks=grid_blocks, workspace=gnm.make_workspace(reg, grid_blocks))
    torch.cuda.synchronize()
    shape = (nw, reg.n_sites)
    return (gnm.acc_to_numpy(acc_s), fl_s.cpu().numpy().reshape(shape),
            gnm.acc_to_numpy(acc_w), fl_w.cpu().numpy().reshape(shape))


def _check(reg, r, rec, off, **kw):
    got, gf, ref, rf = _both(reg, rec, off, **kw)
    assert (got == ref).all(), diff(got, ref)
    assert (gf == rf).all()
    orc = oracle.Registry.from_generated(r)
    exp = orc.classify_aggregate(rec) if off is None else orc.classify_aggregate(rec, window_offsets=off)
    exp = exp if off is not None else exp[None]
    assert (got == exp).all(), diff(got, exp)
    assert (gf == oracle.flags(exp, r.n_sites)).all()


def test_static_scratch_two_calls_second_smaller():
    import torch
    assert torch.cuda.is_available()
    r = flowgen.registry_for(flowgen.PLAIN_SMALL)
    reg = gnm.Registry.from_generated(r)
    assert gnm.static_scratch_bytes() == 32 << 20
    big = flowgen.records_for(flowgen.PLAIN_SMALL, reg=r, n=300_001)
    say("static scratch: call 1, one window of", big.n, "records")
    _check(reg, r, big, None)
    # smaller, several windows, more workgroups than the first call's tables
    small = flowgen.records_for(flowgen.BATCHED, reg=r, n=90_000)
    off = small.window_offsets
    say("static scratch: call 2,", small.n, "records in", len(off) - 1, "windows, 300 workgroups")
    _check(reg, r, small, off, grid_blocks=300)
    say("static scratch: call 3, one window of 5,003 records")
    _check(reg, r, small.slice(0, 5003), None)


def test_static_scratch_large_rows():
    """The 1,000-site registry: 2,003-row tables, 256 of which fill most of the scratch."""
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    reg = gnm.Registry.from_generated(r)
    assert reg.info()["acc_in_lds"] == 1
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r, n=1_500_007)
    say("static scratch: plain-large registry, one window of", rec.n, "records on 256 workgroups")
    _check(reg, r, rec, None, grid_blocks=256)
    part = rec.slice(0, 200_000)
    off = np.array([0, 1, 70_000, 70_000, 200_000], dtype=np.uint64)
    say("static scratch: plain-large registry,", part.n, "records in 4 windows on 64 workgroups")
    _check(reg, r, part, off, grid_blocks=64)


def test_static_scratch_rejections():
    import torch
    r = flowgen.registry_for(flowgen.PLAIN_LARGE)
    reg = gnm.Registry.from_generated(r)
    rec = flowgen.records_for(flowgen.PLAIN_LARGE, reg=r, n=20_000)
    d = to_device(rec)
    acc = torch.full((1, reg.rows, 8), 7, dtype=torch.int64, device=DEV)
    fl = torch.full((reg.n_sites,), 9, dtype=torch.uint8, device=DEV)
    # 600 workgroups x 2,003 rows x 56 bytes pass 32 MiB
    assert gnm.workspace_bytes(reg, 600) > gnm.static_scratch_bytes()
    with pytest.raises(gnm.GnmError) as ei:
        gnm.classify_flag_static(reg, d, acc, fl, n=rec.n, grid_blocks=600)
    assert ei.value.code == gnm.GNM_E_INVAL and "static scratch" in str(ei.value)
    # a caller workspace is refused
    c = gnm.records_struct(d, rec.n)
    ws = gnm.make_workspace(reg)
    p = gnm.make_params(workspace=ws)
    rc = gnm.lib().gnm_classify_flag_static(reg.handle, ctypes.byref(c), None, 1, ctypes.byref(p),
                                            ctypes.c_void_p(acc.data_ptr()), 1_000_000, 0,
                                            ctypes.c_void_p(fl.data_ptr()), gnm._stream_handle(None))
    assert rc == gnm.GNM_E_INVAL
    torch.cuda.synchronize()
    # nothing was enqueued by the refused calls
    assert (acc.cpu().numpy() == 7).all() and (fl.cpu().numpy() == 9).all()

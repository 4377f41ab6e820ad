"""GPU test helpers: upload SoA records, run the library, fetch tables."""
import numpy as np

import paper_1108_1785_amd as gnm

DEV = "cuda:0"


def to_device(rec, device=DEV):
    import torch
    d = {}
    for f in ("src_ip", "dst_ip", "packets", "first_ms", "last_ms"):
        d[f] = torch.from_numpy(np.ascontiguousarray(getattr(rec, f)).view(np.int32)).to(device)
    d["bytes"] = torch.from_numpy(np.ascontiguousarray(rec.bytes).view(np.int64)).to(device)
    return d


def offsets_to_device(off, device=DEV):
    import torch
    return torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(device)


def run(reg, rec, window_offsets=None, bulk_bytes=1_000_000, acc=None, accumulate=False,
        records_per_thread=0, grid_blocks=0, dev_rec=None, workspace=None, shift=0, **params):
    """Classify/aggregate a host Records run on the GPU; returns uint64 [n_windows?, rows, 8].

    shift > 0 offsets every field pointer by that many records (misaligned
    views); params go to gnm.classify_aggregate (e.g. flush_records)."""
    import torch
    off = window_offsets if window_offsets is not None else rec.window_offsets
    nw = 1 if off is None else len(off) - 1
    if dev_rec is not None:
        d = dev_rec
    elif shift:
        import flowgen
        pad = flowgen.concat([rec.slice(0, shift), rec]) if rec.n >= shift else None
        full = to_device(pad)
        d = {f: t[shift:] for f, t in full.items()}
    else:
        d = to_device(rec)
    if acc is None:
        acc = torch.empty((nw, reg.rows, 8), dtype=torch.int64, device=DEV)
    doff = None if off is None else offsets_to_device(off)
    gnm.classify_aggregate(reg, d, acc, window_offsets=doff, n_windows=nw, bulk_bytes=bulk_bytes,
                           accumulate=accumulate, records_per_thread=records_per_thread,
                           grid_blocks=grid_blocks, n=rec.n, workspace=workspace, **params)
    torch.cuda.synchronize()
    out = gnm.acc_to_numpy(acc)
    return out[0] if off is None else out


def flags(reg, acc_np, threshold_bps=1_000_000, min_bulk_flows=0):
    import torch
    a = acc_np if acc_np.ndim == 3 else acc_np[None]
    nw = a.shape[0]
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(DEV)
    f = torch.empty(nw * reg.n_sites, dtype=torch.uint8, device=DEV)
    gnm.flag_suboptimal(reg, t, nw, f, threshold_bps, min_bulk_flows)
    torch.cuda.synchronize()
    out = f.cpu().numpy().reshape(nw, reg.n_sites)
    return out if acc_np.ndim == 3 else out[0]


def diff(got, exp, limit=5):
    """Human-readable first mismatches (rows, fields)."""
    bad = np.argwhere(got != exp)
    return ["idx=%s got=%d exp=%d" % (tuple(i), int(got[tuple(i)]), int(exp[tuple(i)])) for i in bad[:limit]]

"""GPU parity of the NetFlow v5 decode step against the CPU oracle decoder:
every field of every record, the record and rejection totals, bit for bit;
and decode followed by classify/aggregate against the oracle's tables."""
import sys

import numpy as np
import pytest

import flowgen
import oracle
import paper_1108_1785_amd as gnm
from oracle import netflow
from tests._gpu import DEV, diff
from tests._helpers import load_golden

pytestmark = pytest.mark.gpu
FIELDS = ("src_ip", "dst_ip", "src_port", "dst_port", "proto", "bytes", "packets", "first_ms", "last_ms")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_decode(buf, off, capacity=None, ports=True):
    import torch
    d_buf = torch.from_numpy(np.ascontiguousarray(buf)).to(DEV)
    d_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(DEV)
    cap = capacity if capacity is not None else max(1, 30 * (len(off) - 1))
    out = gnm.make_records_out(cap, device=DEV, ports=ports)
    for t in out.values():
        t.fill_(-1 if t.dtype != torch.uint8 else 255)
    counts = gnm.netflow_v5_decode(d_buf, d_off, out)
    torch.cuda.synchronize()
    n_rec, n_rej = (int(x) for x in counts.cpu().numpy())
    host = {f: t.cpu().numpy() for f, t in out.items()}
    typ = {"src_port": np.uint16, "dst_port": np.uint16, "proto": np.uint8, "bytes": np.uint64}
    host = {f: v.view(typ.get(f, np.uint32)) for f, v in host.items()}
    return host, n_rec, n_rej, out


def check(host, exp, n, fields=FIELDS):
    for f in fields:
        g, e = host[f][:n], exp[f][:n]
        bad = np.nonzero(g != e)[0]
        assert bad.size == 0, (f, [(int(i), int(g[i]), int(e[i])) for i in bad[:5]])


def test_golden_datagram(torch_cuda):
    say("case: ingest golden datagram")
    g = load_golden("netflow_v5.json")
    buf = np.frombuffer(bytes.fromhex("".join(g["header"]) + "".join("".join(r) for r in g["records"])),
                        dtype=np.uint8).copy()
    off = np.array([0, buf.size], dtype=np.uint64)
    host, n_rec, n_rej, _ = gpu_decode(buf, off)
    exp, rej = netflow.decode_netflow_v5(buf, off)
    assert (n_rec, n_rej) == (2, 0) and rej == 0
    check(host, exp, 2)


@pytest.mark.parametrize("n,malformed,seed", [(1, 0, 1), (29, 0, 2), (30, 0, 3), (31, 5, 4), (20_000, 0, 5),
                                              (20_000, 300, 6), (100_003, 40, 7)])
def test_decode_matches_oracle(torch_cuda, n, malformed, seed):
    say("case: ingest", n, "records,", malformed, "malformed datagrams")
    rec = flowgen.v5_records(flowgen.PLAIN_SMALL, n, stream=seed)
    buf, off = flowgen.encode_netflow_v5(rec, np.random.default_rng(seed), malformed=malformed)
    exp, rej = netflow.decode_netflow_v5(buf, off)
    host, n_rec, n_rej, _ = gpu_decode(buf, off)
    assert (n_rec, n_rej) == (exp["src_ip"].size, rej) == (n, malformed)
    check(host, exp, n)


def test_capacity_and_optional_fields(torch_cuda):
    say("case: ingest capacity below the record count; no ports/proto")
    rec = flowgen.v5_records(flowgen.PLAIN_SMALL, 5_000, stream=9)
    buf, off = flowgen.encode_netflow_v5(rec, np.random.default_rng(9), malformed=7)
    exp, _ = netflow.decode_netflow_v5(buf, off)
    host, n_rec, n_rej, _ = gpu_decode(buf, off, capacity=1_234, ports=False)
    assert (n_rec, n_rej) == (5_000, 7)
    check(host, exp, 1_234, fields=("src_ip", "dst_ip", "bytes", "packets", "first_ms", "last_ms"))
    assert "src_port" not in host


def test_empty_and_out_of_buffer_offsets(torch_cuda):
    import torch
    say("case: ingest with no datagrams; offsets past the buffer")
    host, n_rec, n_rej, _ = gpu_decode(np.zeros(16, dtype=np.uint8), np.array([0], dtype=np.uint64), capacity=4)
    assert (n_rec, n_rej) == (0, 0)
    g = load_golden("netflow_v5.json")
    one = bytes.fromhex("".join(g["header"]) + "".join("".join(r) for r in g["records"]))
    buf = np.frombuffer(one + one, dtype=np.uint8).copy()
    off = np.array([0, 120, 10**12], dtype=np.uint64)  # the second span runs past the buffer: rejected
    host, n_rec, n_rej, _ = gpu_decode(buf, off)
    assert (n_rec, n_rej) == (2, 1)
    with pytest.raises(gnm.GnmError):
        d = torch.from_numpy(np.concatenate([np.zeros(4, np.uint8), buf])).to(DEV)
        gnm.netflow_v5_decode(d[1:], torch.zeros(2, dtype=torch.int64, device=DEV),
                              gnm.make_records_out(4, device=DEV))


def test_full_size_decode_then_classify(torch_cuda):
    """10,000,000 records in 333,334+ datagrams: decode, then classify the
    decoded window and compare the tables with the oracle's."""
    import torch
    say("case: ingest 10M records (plain-large recipe), then classify")
    rec = flowgen.v5_records(flowgen.PLAIN_LARGE, 10_000_000, stream=1)
    buf, off = flowgen.encode_netflow_v5(rec, np.random.default_rng(11), malformed=100)
    host, n_rec, n_rej, out = gpu_decode(buf, off, capacity=10_000_000)
    assert (n_rec, n_rej) == (10_000_000, 100)
    # the oracle on 2,000 sampled datagrams, one at a time, at their output positions
    first = np.concatenate([[0], np.cumsum([netflow.datagram_count(buf, int(off[d]), int(off[d + 1]))
                                            for d in range(len(off) - 1)])])
    rng = np.random.default_rng(12)
    for d in sorted(set(int(x) for x in rng.integers(0, len(off) - 1, size=2000)) | {0, len(off) - 2}):
        e, _ = netflow.decode_netflow_v5(buf, off[d:d + 2] - np.uint64(0))
        lo = int(first[d])
        for f in FIELDS:
            assert np.array_equal(host[f][lo:lo + e[f].size], e[f]), (d, f)
    # and every record equals the one it was encoded from (decode inverts the
    # generator's encoder, a round trip the CPU pins establish)
    for f in FIELDS:
        assert np.array_equal(host[f], getattr(rec, f)), f
    reg_h = flowgen.registry_for(flowgen.PLAIN_LARGE)
    reg = gnm.Registry.from_generated(reg_h)
    acc = torch.empty((1, reg.rows, 8), dtype=torch.int64, device=DEV)
    gnm.classify_aggregate(reg, out, acc, n=10_000_000, workspace=gnm.make_workspace(reg))
    torch.cuda.synchronize()
    got = gnm.acc_to_numpy(acc)[0]
    want = oracle.Registry.from_generated(reg_h).classify_aggregate(rec)
    assert (got == want).all(), diff(got, want)

"""Pins of the NetFlow v5 decode oracle (CPU only): a hand-built datagram,
the paper's sizes, a round trip through the generator's independent encoder,
and every kind of malformed datagram."""
import numpy as np
import pytest

import flowgen
from oracle import netflow
from tests._helpers import ip, load_golden


def _golden_datagram():
    g = load_golden("netflow_v5.json")
    hexs = "".join(g["header"]) + "".join("".join(r) for r in g["records"])
    return np.frombuffer(bytes.fromhex(hexs), dtype=np.uint8), g


def test_golden_datagram():
    buf, g = _golden_datagram()
    assert buf.size == 24 + 2 * 48
    out, rejected = netflow.decode_netflow_v5(buf, np.array([0, buf.size], dtype=np.uint64))
    assert rejected == 0
    for k, exp in enumerate(g["expected"]):
        for f, v in exp.items():
            want = ip(v) if f in ("src_ip", "dst_ip") else v
            assert int(out[f][k]) == want, (k, f)


def test_paper_sizes():
    # 48-byte records; 30 of them and the header fit a 1500-byte Ethernet
    # frame's UDP payload (1500 - 20 IP - 8 UDP), 31 do not (§IV.A.3)
    assert netflow.RECORD.size == 48 and netflow.HEADER.size == 24
    assert 24 + 30 * 48 <= 1500 - 28 < 24 + 31 * 48


def test_round_trip_through_the_encoder():
    rec = flowgen.v5_records(flowgen.PLAIN_SMALL, 20_000)
    buf, off = flowgen.encode_netflow_v5(rec, np.random.default_rng(3))
    out, rejected = netflow.decode_netflow_v5(buf, off)
    assert rejected == 0
    for f in ("src_ip", "dst_ip", "src_port", "dst_port", "proto", "bytes", "packets", "first_ms", "last_ms"):
        assert np.array_equal(out[f], getattr(rec, f)), f


def test_malformed_datagrams_rejected():
    rec = flowgen.v5_records(flowgen.PLAIN_SMALL, 3_000)
    rng = np.random.default_rng(8)
    buf, off = flowgen.encode_netflow_v5(rec, rng, malformed=60)
    out, rejected = netflow.decode_netflow_v5(buf, off)
    assert rejected == 60
    assert np.array_equal(out["src_ip"], rec.src_ip) and np.array_equal(out["last_ms"], rec.last_ms)


@pytest.mark.parametrize("mutate,accepted", [
    (lambda b: b, True),
    (lambda b: b[:-1], False),                       # one byte short of the second record
    (lambda b: b + b"\0" * 7, True),                 # trailing bytes are ignored
    (lambda b: b"\x00\x09" + b[2:], False),          # version 9
    (lambda b: b[:2] + b"\x00\x00" + b[4:], False),  # count 0
    (lambda b: b[:2] + b"\x00\x1f" + b[4:], False),  # count 31
    (lambda b: b[:23], False),                       # shorter than the header
])
def test_acceptance_rule(mutate, accepted):
    buf, _ = _golden_datagram()
    b = mutate(buf.tobytes())
    arr = np.frombuffer(b, dtype=np.uint8)
    out, rejected = netflow.decode_netflow_v5(arr, np.array([0, arr.size], dtype=np.uint64))
    assert rejected == (0 if accepted else 1)
    assert out["src_ip"].size == (2 if accepted else 0)


def test_misaligned_start_rejected():
    buf, _ = _golden_datagram()
    b = np.frombuffer(b"\0\0" + buf.tobytes(), dtype=np.uint8)
    out, rejected = netflow.decode_netflow_v5(b, np.array([0, 2, b.size], dtype=np.uint64))
    assert rejected == 2 and out["src_ip"].size == 0  # a 2-byte stub and a datagram at offset 2

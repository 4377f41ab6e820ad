"""CPU oracle of the NetFlow v5 decode step (test infrastructure only).

Turns router export datagrams into the structure-of-arrays records the
classify path reads.  The paper's routers export NetFlow V5 over UDP: 48-byte
records, at most 30 per 1500-byte datagram (§III.B.1, FlowData Receiver
Thread; §IV.A.3).  The field layout is the public NetFlow version 5 export
format, every field big-endian: a 24-byte header (version, count, sys_uptime,
unix_secs, unix_nsecs, flow_sequence, engine_type, engine_id,
sampling_interval) and 48-byte records (srcaddr, dstaddr, nexthop, input,
output, dPkts, dOctets, First, Last, srcport, dstport, pad1, tcp_flags, prot,
tos, src_as, dst_as, src_mask, dst_mask, pad2).

A datagram d spans buf[offsets[d], offsets[d+1]).  It is accepted when its
start is a multiple of 4, it holds the 24-byte header, the version is 5, the
count is 1..30 and the span holds count records; bytes past them are
ignored.  Records of accepted datagrams are emitted in datagram order;
rejected datagrams are counted.  Each datagram is parsed on its own with
`struct`, one record at a time.
"""
from __future__ import annotations

import struct

import numpy as np

HEADER = struct.Struct(">HHIIIIBBH")             # 24 bytes
RECORD = struct.Struct(">IIIHHIIIIHHBBBBHHBBH")  # 48 bytes
MAX_RECORDS = 30


def datagram_count(buf, start: int, end: int) -> int:
    """Records an accepted datagram carries, or 0 when it is rejected."""
    if end < start or end - start < HEADER.size or start % 4:
        return 0
    version, count = struct.unpack_from(">HH", buf, start)
    if version != 5 or not 1 <= count <= MAX_RECORDS or end - start < HEADER.size + RECORD.size * count:
        return 0
    return count


def decode_netflow_v5(buf: np.ndarray, offsets: np.ndarray):
    """(dict of SoA arrays, n_rejected).  Fields: src_ip, dst_ip, src_port,
    dst_port, proto, bytes (u64, from the 32-bit dOctets), packets, first_ms,
    last_ms."""
    mv = memoryview(np.ascontiguousarray(buf, dtype=np.uint8))
    off = [int(x) for x in offsets]
    cols = {k: [] for k in ("src_ip", "dst_ip", "src_port", "dst_port", "proto", "bytes", "packets",
                            "first_ms", "last_ms")}
    rejected = 0
    for d in range(len(off) - 1):
        c = datagram_count(mv, off[d], off[d + 1])
        if c == 0:
            rejected += 1
            continue
        body = mv[off[d] + HEADER.size: off[d] + HEADER.size + RECORD.size * c]
        for (src, dst, _nexthop, _inp, _outp, pkts, octets, first, last, sport, dport, _pad1, _flags, prot,
             _tos, _sas, _das, _smask, _dmask, _pad2) in RECORD.iter_unpack(body):
            cols["src_ip"].append(src)
            cols["dst_ip"].append(dst)
            cols["src_port"].append(sport)
            cols["dst_port"].append(dport)
            cols["proto"].append(prot)
            cols["bytes"].append(octets)
            cols["packets"].append(pkts)
            cols["first_ms"].append(first)
            cols["last_ms"].append(last)
    types = {"src_port": np.uint16, "dst_port": np.uint16, "proto": np.uint8, "bytes": np.uint64}
    out = {k: np.array(v, dtype=types.get(k, np.uint32)) for k, v in cols.items()}
    return out, rejected

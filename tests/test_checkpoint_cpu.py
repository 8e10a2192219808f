"""Checkpoint file format (isdf_save / isdf_load), checked on the host.

The writer below builds files from the format stated in include/isdf.h
(144-byte little-endian header, payload of interpolation points, factor
ranks, X^k, Pi^q and W^q of one q per class {q, -q}, FNV-1a 64 checksum)
without the library; isdf_load must reject every malformed variant before
any device call (ISDF_E_INVALID, no context).  A well-formed file passes
the host checks: on a machine without a GPU the load then stops at the
device (ISDF_E_DEVICE)."""
import ctypes
import struct

import numpy as np
import pytest

import paper_2601_16379_amd as pkg

ISDF_OK, ISDF_E_INVALID, ISDF_E_DEVICE = 0, -1, -5


def fnv1a64(data):
    h = 1469598103934665603
    for b in data:
        h ^= b
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def n_classes(kmesh):
    """Classes {q, -q}: q whose -q (mesh negation) is not smaller."""
    m1, m2, m3 = kmesh
    n = 0
    for j1 in range(m1):
        for j2 in range(m2):
            for j3 in range(m3):
                q = (j1 * m2 + j2) * m3 + j3
                mq = (((-j1) % m1) * m2 + (-j2) % m2) * m3 + (-j3) % m3
                n += mq >= q
    return n


def build(grid=(6, 6, 6), kmesh=(2, 1, 3), n_orb=2, n_ip=5, **over):
    nk = int(np.prod(kmesh))
    nh = over.get("nh", n_classes(kmesh))
    rng = np.random.default_rng(0)
    ip = over.get("ip", np.arange(0, 3 * n_ip, 3, dtype=np.int32))
    rank = over.get("rank", np.full(nh, n_ip, dtype=np.int32))
    x = rng.standard_normal(2 * nk * n_orb * n_ip)
    pi = rng.standard_normal(2 * nh * n_ip * n_ip)
    w = rng.standard_normal(2 * nh * n_ip * n_ip)
    payload = (np.asarray(ip, np.int32).tobytes() + np.asarray(rank, np.int32).tobytes()
               + x.tobytes() + pi.tobytes() + w.tobytes())
    payload_bytes = over.get("payload_bytes", len(payload))
    checksum = over.get("checksum", fnv1a64(payload))
    head = (over.get("magic", b"ISDFCKP1") + struct.pack("<II", over.get("version", 1), 144)
            + struct.pack("<9i", *grid, *kmesh, n_orb, n_ip, nh) + struct.pack("<I", 0)
            + struct.pack("<9d", *np.eye(3).reshape(-1) * 5.0) + struct.pack("<QQ", payload_bytes, checksum))
    assert len(head) == 144
    return head + payload


def load(path):
    lib = pkg.load_library()
    h = ctypes.c_void_p()
    st = lib.isdf_load(ctypes.byref(h), str(path).encode(), None)
    msg = lib.isdf_last_error(None).decode()
    if st == ISDF_OK:
        lib.isdf_destroy(h)
    else:
        assert not h.value
    return st, msg


def test_wellformed_file_passes_host_checks(tmp_path):
    p = tmp_path / "ok.ckp"
    p.write_bytes(build())
    st, msg = load(p)
    assert st in (ISDF_OK, ISDF_E_DEVICE), msg


@pytest.mark.parametrize("case,data,needle", [
    ("magic", dict(magic=b"ISDFCKP0"), "not an isdf checkpoint"),
    ("version", dict(version=2), "version"),
    ("classes", dict(nh=5), "k mesh"),
    ("length", dict(payload_bytes=10), "k mesh"),
    ("checksum", dict(checksum=12345), "checksum"),
    ("rank", dict(rank=np.array([5, 5, 6, 5], np.int32)), "rank"),
    ("duplicate ip", dict(ip=np.array([0, 3, 3, 9, 12], np.int32)), "duplicate"),
    ("ip range", dict(ip=np.array([0, 3, 6, 9, 216], np.int32)), "range"),
])
def test_malformed_files_are_refused(tmp_path, case, data, needle):
    assert n_classes((2, 1, 3)) == 4
    p = tmp_path / "bad.ckp"
    p.write_bytes(build(**data))
    st, msg = load(p)
    assert st == ISDF_E_INVALID and needle in msg, (case, st, msg)


def test_truncated_and_trailing_and_missing(tmp_path):
    good = build()
    for name, data, needle in [("trunc_head", good[:100], "header"), ("trunc_body", good[:-8], "truncated"),
                               ("trailing", good + b"\0", "trailing")]:
        p = tmp_path / name
        p.write_bytes(data)
        st, msg = load(p)
        assert st == ISDF_E_INVALID and needle in msg, (name, msg)
    st, msg = load(tmp_path / "absent.ckp")
    assert st == ISDF_E_INVALID and "cannot open" in msg

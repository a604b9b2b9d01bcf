"""Binary particle snapshots (adm1_snapshot_*, host code, no GPU needed)
against an independent numpy reading and writing of the documented layout:
bit-exact round trips both ways, field subsets, strided rows, errors."""
from __future__ import annotations

import os

import numpy as np
import pytest

from paper_2311_08927_amd import snapshot as S


def numpy_write(path, n, time_s, fields):
    """The documented layout, written with numpy alone."""
    mask = 0
    body = []
    for bit, arr in fields:
        if arr is not None:
            mask |= bit
            body.append(np.ascontiguousarray(arr[..., :n]))
    hdr = np.zeros(64, np.uint8)
    hdr[:8] = np.frombuffer(b"ADM1SNAP", np.uint8)
    hdr[8:12] = np.frombuffer(np.uint32(1).tobytes(), np.uint8)
    hdr[12:16] = np.frombuffer(np.uint32(mask).tobytes(), np.uint8)
    hdr[16:24] = np.frombuffer(np.uint64(n).tobytes(), np.uint8)
    hdr[24:32] = np.frombuffer(np.float64(time_s).tobytes(), np.uint8)
    with open(path, "wb") as fh:
        fh.write(hdr.tobytes())
        for a in body:
            fh.write(a.tobytes())


def numpy_read(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"ADM1SNAP"
    ver, mask = np.frombuffer(raw[8:16], np.uint32)
    n = int(np.frombuffer(raw[16:24], np.uint64)[0])
    t = float(np.frombuffer(raw[24:32], np.float64)[0])
    assert ver == 1 and raw[32:64] == bytes(32)
    off, out = 64, {}
    for bit, rows, dt in ((1, 3, np.float32), (2, 3, np.float32), (4, 1, np.float32),
                          (8, 35, np.float64)):
        if mask & bit:
            k = rows * n * np.dtype(dt).itemsize
            out[bit] = np.frombuffer(raw[off:off + k], dt).reshape(rows, n)
            off += k
    assert off == len(raw)
    return n, int(mask), t, out


def arrays(n, ld, seed):
    g = np.random.default_rng(seed)
    pos = g.random((3, ld), dtype=np.float32)
    vel = g.standard_normal((3, ld)).astype(np.float32)
    rho = (1000 + g.random(ld)).astype(np.float32)
    state = g.random((35, ld))
    state[3, 5] = np.nan  # payloads travel bit for bit
    return pos, vel, rho, state


@pytest.mark.parametrize("n,ld", [(1000, 1024), (3_000_000, 3_000_064)])
def test_library_write_numpy_read(tmp_path, n, ld):
    pos, vel, rho, state = arrays(n, ld, 1)
    p = str(tmp_path / "a.bin")
    S.adm1_snapshot_write(p, n, ld, 12.5, pos, vel, rho, state)
    m, mask, t, out = numpy_read(p)
    assert (m, mask, t) == (n, 15, 12.5)
    for bit, a in ((1, pos), (2, vel), (4, rho.reshape(1, -1)), (8, state)):
        assert out[bit].tobytes() == np.ascontiguousarray(a[..., :n]).tobytes()
    assert S.adm1_snapshot_info(p) == (n, 15, 12.5)


def test_numpy_write_library_read_subsets(tmp_path):
    n, ld = 777, 832
    pos, vel, rho, state = arrays(n, ld, 2)
    p = str(tmp_path / "b.bin")
    numpy_write(p, n, 3.0, [(1, pos), (2, None), (4, rho), (8, state)])
    assert S.adm1_snapshot_info(p) == (n, 13, 3.0)
    # all present fields
    bp, br, bs = np.zeros((3, ld), np.float32), np.zeros(ld, np.float32), np.zeros((35, ld))
    assert S.adm1_snapshot_read(p, ld, pos=bp, rho=br, state=bs) == n
    assert bp[:, :n].tobytes() == pos[:, :n].tobytes()
    assert br[:n].tobytes() == rho[:n].tobytes()
    assert bs[:, :n].tobytes() == state[:, :n].tobytes()
    # one field skipped
    bs2 = np.zeros((35, ld))
    assert S.adm1_snapshot_read(p, ld, state=bs2) == n
    assert bs2[:, :n].tobytes() == state[:, :n].tobytes()
    # a requested field that is absent
    assert S.adm1_snapshot_read(p, ld, vel=np.zeros((3, ld), np.float32), check=False) == -10


def test_errors(tmp_path):
    p = str(tmp_path / "c.bin")
    pos = np.zeros((3, 128), np.float32)
    assert S.adm1_snapshot_write(p, 200, 128, 0.0, pos, check=False) == -2
    assert S.adm1_snapshot_write(str(tmp_path / "no" / "x.bin"), 10, 128, 0.0, pos,
                                 check=False) == -10
    S.adm1_snapshot_write(p, 100, 128, 0.0, pos)
    assert S.adm1_snapshot_read(p, 64, pos=np.zeros((3, 64), np.float32), check=False) == -2
    assert S.adm1_snapshot_read(str(tmp_path / "missing.bin"), 128, pos=pos, check=False) == -10
    raw = bytearray(open(p, "rb").read())
    open(p, "wb").write(bytes(raw[:-4]))          # truncated
    assert S.adm1_snapshot_read(p, 128, pos=pos, check=False) == -10
    raw[0] = ord("X")
    open(p, "wb").write(bytes(raw))                # bad magic
    assert S.adm1_snapshot_read(p, 128, pos=pos, check=False) == -10
    assert S.adm1_snapshot_write(p, 0, 1, 0.0) == 0   # empty snapshot
    assert S.adm1_snapshot_info(p) == (0, 0, 0.0)
    os.remove(p)


def test_binding_rejects_buffers_that_do_not_fit(tmp_path):
    """The C routines move rows x ld elements at offsets r x ld without
    knowing the buffers' sizes: the binding refuses a buffer of the wrong
    element type, shape, size or memory order before the call."""
    import torch
    p = str(tmp_path / "s.bin")
    ld, n = 128, 100
    pos = np.zeros((3, ld), np.float32)
    state = np.zeros((35, ld), np.float64)
    S.adm1_snapshot_write(p, n, ld, 0.0, pos, state=state)
    bad = [
        dict(state=np.zeros((35, ld), np.float32)),            # wrong dtype
        dict(state=np.zeros((35, 2 * ld), np.float64)),        # row stride != ld
        dict(state=np.zeros((34, ld), np.float64)),            # too few rows
        dict(state=np.zeros((35 * ld - 1,), np.float64)),      # flat and too short
        dict(pos=np.zeros((ld, 3), np.float32).T),             # not C-contiguous
        dict(pos=torch.zeros((3, ld), dtype=torch.float64)),   # torch, wrong dtype
        dict(rho=np.zeros(ld - 1, np.float32)),                # too short
    ]
    for kw in bad:
        with pytest.raises(ValueError):
            S.adm1_snapshot_read(p, ld, **kw)
    ro = np.zeros((3, ld), np.float32)
    ro.flags["WRITEABLE"] = False
    with pytest.raises(ValueError):
        S.adm1_snapshot_read(p, ld, pos=ro)
    with pytest.raises(ValueError):
        S.adm1_snapshot_write(p, n, ld, 0.0, state=np.zeros((35, 64), np.float64))
    # fitting buffers, numpy and CPU torch, flat or [rows][ld], still pass
    assert S.adm1_snapshot_read(p, ld, pos=torch.zeros((3, ld), dtype=torch.float32),
                                state=np.zeros(35 * ld, np.float64)) == n

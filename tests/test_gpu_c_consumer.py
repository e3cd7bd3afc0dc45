"""A plain C program (tests/c/consumer.c) drives the library through the C
ABI alone -- load, crater edit, renders in every exact mode into device
memory it allocates itself -- and its hit records match the oracle's render
of the same map with the oracle's own crater edit."""
import os
import subprocess

import numpy as np
import pytest

import oracle

from test_abi_cpu import build_c_consumer
from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def test_c_program_matches_oracle(tmp_path):
    exe = build_c_consumer(str(tmp_path / "consumer"))
    out = str(tmp_path / "hits.bin")
    r = subprocess.run([exe, out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(out, "rb").read()
    W, H, nv = np.frombuffer(raw[:12], np.int32)
    off = 12
    planes = []
    for _ in range(3):
        planes.append(np.frombuffer(raw[off:off + W * H], np.uint8).reshape(H, W))
        off += W * H
    x0, y0, size, depth = (int(x) for x in np.frombuffer(raw[off:off + 16], np.int32))
    off += 16
    views = np.frombuffer(raw[off:off + 84 * nv], oracle.VIEW_DT)
    off += 84 * nv
    rays = int((views["width"].astype(np.int64) * views["height"]).sum())
    hits = np.frombuffer(raw[off:off + 8 * rays], np.uint32).reshape(rays, 2)
    assert off + 8 * rays == len(raw)
    F, B, T = oracle.apply_edits(*planes, [dict(kind=oracle.EDIT_CRATER, x0=x0, y0=y0, w=size,
                                                h=size, depth=depth)])
    assert oracle.valid_columns(F, B, T)
    wo, do = oracle.render(F, B, T, list(views))
    assert_parity(hits[:, 0].copy(), hits[:, 1].copy().view(np.float32), wo, do, "C consumer")
    assert np.mean(wo != oracle.MISS) > 0.5

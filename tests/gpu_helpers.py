"""Shared helpers for the GPU parity tests (inputs go to the device, results come back as numpy)."""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2005_01372_amd import lsop


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(lsop.LIB_PATH):
        pytest.fail("liblsop.so is not built: GPU tests need the HIP library (run the build first)")
    lsop.load_library()


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def make_op(w, dtype=lsop.C128, max_vec=16):
    op = lsop.Operator(w.nx, w.nz, dtype, max_vec)
    op.set_problem(torch.as_tensor(w.vel).cuda(), w.h, w.freq, w.c0)
    return op


def golden_layered_salt():
    """The oracle's solution of the 256^2 layered + salt workload at sampled cells (tests/golden/, written by
    make_layered_salt_256.py from oracle/ only)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "layered_salt_256_solution.txt")
    norms, cells = {}, {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "R":
            norms[int(f[1])] = float(f[4])
        else:
            cells.setdefault(int(f[1]), []).append((int(f[2]), int(f[3]), complex(float(f[4]), float(f[5]))))
    return norms, cells

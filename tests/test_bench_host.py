"""Host-side checks of bench.py's marshalling (no GPU): the pfm_problem
records it builds by hand must have the binding's layout, field for field."""

import ctypes
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from paper_2210_03714_amd import pfm  # noqa: E402


def test_problem_dtype_matches_binding():
    dt = bench.problem_dtype(np)
    assert dt.itemsize == ctypes.sizeof(pfm.Problem)
    assert set(dt.names) == {f for f, _ in pfm.Problem._fields_}


def test_problem_array_pointers_and_strides():
    A = torch.zeros(3, 5, 5, dtype=torch.float64)
    F = torch.zeros(3, 5, 7, dtype=torch.float64)   # padded leading dimension
    arr = bench._problem_array(np, A, {"F_exp": F}, F.stride(1))
    recs = (pfm.Problem * 3).from_buffer_copy(arr.tobytes())
    for b in range(3):
        r = recs[b]
        assert (r.n, r.p, r.lda, r.ldf) == (5, 0, 5, 7)
        assert r.A == A.data_ptr() + b * 25 * 8
        assert r.F_exp == F.data_ptr() + b * 35 * 8
        assert not r.F_phi1 and not r.F_phi2 and not r.V

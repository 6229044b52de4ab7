"""The measurement probes (fgs_probe) run, report the work of their launch
and leave finite checksums; an unknown kind is refused."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_probes_run_and_report_their_work():
    from paper_2604_01844_amd import _abi as A
    L = A.lib()
    blocks, iters = 8, 4
    sink = torch.full((blocks * 256,), float("nan"), device="cuda")
    threads = blocks * 256
    expect = {0: threads * iters * 64.0, 1: threads * iters * 32.0, 2: threads * iters * 32.0,
              3: threads * iters * 64.0, 4: threads * iters * 128.0, 5: threads / 64 * iters * 4 * 32768.0}
    for kind, work in expect.items():
        w = ctypes.c_double()
        A.check(L.fgs_probe(kind, blocks, iters, A.ptr(sink), ctypes.byref(w), A.stream_ptr()))
        torch.cuda.synchronize()
        assert w.value == work, kind
        assert bool(torch.isfinite(sink).all()), kind
    w = ctypes.c_double()
    assert L.fgs_probe(6, blocks, iters, A.ptr(sink), ctypes.byref(w), A.stream_ptr()) == A.FGS_E_INVALID
    assert L.fgs_probe(0, 0, iters, A.ptr(sink), ctypes.byref(w), A.stream_ptr()) == A.FGS_E_INVALID

"""The benchmark's calibration probe (the dense solver's access pattern
without its arithmetic, in its own library outside the C-ABI) runs and
leaves its sink alone."""
import os
import sys

import pytest
import torch

from gpu_helpers import lib

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stream_probe_runs_and_checks_arguments():
    d = lib()
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    probe = bench.probe_lib()
    buf = torch.empty(8 * 4096, dtype=torch.uint8, device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert probe.dtm_stream_probe(buf.data_ptr(), 4096, 8, 3, sink.data_ptr(), s) == d.DTM_OK
    torch.cuda.synchronize()
    assert sink.item() == 7.0
    assert probe.dtm_stream_probe(buf.data_ptr(), 4095, 8, 3, sink.data_ptr(), s) == d.DTM_EINVAL
    assert probe.dtm_stream_probe(buf.data_ptr(), 4096, 0, 3, sink.data_ptr(), s) == d.DTM_EINVAL
    assert probe.dtm_stream_probe(None, 4096, 8, 3, sink.data_ptr(), s) == d.DTM_EINVAL

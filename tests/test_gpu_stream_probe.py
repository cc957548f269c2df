"""GPU check of the streaming calibration entry point (kb_stream_probe)."""
import pytest

from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    need_gpu()
    import torch
    return torch


def test_stream_probe_writes_the_sum_of_its_inputs(torch):
    """kb_stream_probe: out_j = sum of the nin inputs element-wise, for
    every output array, and a positive time."""
    import ctypes as C
    import paper_2501_09398_amd as kb
    announce("stream probe output")
    n, nin, nout = 4096, 3, 2
    ws = torch.zeros((nin + nout) * n + 64, dtype=torch.float32, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    off = (base - ws.data_ptr()) // 4
    ins = [torch.arange(n, dtype=torch.float32, device="cuda") * (k + 1) for k in range(nin)]
    for k in range(nin):
        ws[off + k * n: off + (k + 1) * n] = ins[k]
    torch.cuda.synchronize()
    sec = C.c_double()
    rc = kb.lib().kb_stream_probe(nin, nout, n, C.c_void_p(base), (nin + nout) * n * 4, None, 2, C.byref(sec))
    assert rc == 0 and sec.value > 0
    ref = ins[0] + ins[1] + ins[2]
    for j in range(nout):
        got = ws[off + (nin + j) * n: off + (nin + j + 1) * n]
        assert torch.equal(got, ref)

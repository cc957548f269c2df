"""kb_reduce_noalloc against kb_reduce on the same data.

kb_reduce_noalloc runs the deterministic two-pass reduction of kb_reduce
(same kernels, same chunks, same summation order) on caller arrays, with
its per-block partials in the library's static device array instead of a
problem's workspace.  On the same arrays and element count both give the
same bits.  Two calls in a row on the one GPU, the second smaller, check
that the shared array carries nothing from one call into the next.
"""
import numpy as np
import pytest

from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def test_noalloc_sum_equals_kb_reduce(kb):
    """Sum of T of a 2D thermal problem: 300 x 257 (76 chunks of 1024
    cells, a ragged last one), then 40 x 33 (one partial chunk)."""
    import torch
    for shape, seed in (((300, 257), 3), ((40, 33), 4)):
        announce(f"kb_reduce_noalloc sum {shape}")
        with kb.Problem(kb.HEAT2D, shape, kb.HEAT_COEFFS, seed) as p:
            p.run(5, 0)
            ref = p.reduce()[0]
            T = torch.empty(shape, dtype=torch.float32, device="cuda")
            p.read_device(kb.F_T, T)
        out = kb.reduce_noalloc([T])
        torch.cuda.synchronize()
        got = float(out.item())
        print(f"{shape}: noalloc {got!r} kb_reduce {ref!r}")
        assert got == ref


def test_noalloc_energy_equals_kb_reduce(kb):
    """E.E and H.H of an FDTD cavity (three arrays each): kb_reduce sums the
    device layout, rows of N+1 nodes padded with zeros to a multiple of 4
    floats; the same padded arrays handed to kb_reduce_noalloc give the
    same bits.  N = 20, then the smaller N = 6."""
    import torch
    for N in (20, 6):
        announce(f"kb_reduce_noalloc energy N={N}")
        M = N + 1
        pitch = (M + 3) // 4 * 4
        rng = np.random.default_rng(N)
        with kb.Problem(kb.FDTD3D, (N, 64), (0.5, 0.0, 80.0), 0) as p:
            for fid in kb.FDTD_FIELDS.values():
                p.write(fid, rng.standard_normal((M, M, M)).astype(np.float32))
            p.run(3, 0)
            e2, h2 = p.reduce()
            dense = {k: p.read(fid) for k, fid in kb.FDTD_FIELDS.items()}
        padded = {}
        for k, v in dense.items():
            a = np.zeros((M, M, pitch), np.float32)
            a[:, :, :M] = v
            padded[k] = torch.from_numpy(a).cuda()
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        kb.reduce_noalloc([padded[k] for k in ("Ex", "Ey", "Ez")], square=True, out=out[0:1])
        kb.reduce_noalloc([padded[k] for k in ("Hx", "Hy", "Hz")], square=True, out=out[1:2])
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"N={N}: noalloc {got[0]!r} {got[1]!r}, kb_reduce {e2!r} {h2!r}")
        assert got[0] == e2 and got[1] == h2


def test_noalloc_rejects_bad_arguments(kb):
    import torch
    x = torch.zeros(8, dtype=torch.float32, device="cuda")
    with pytest.raises(kb.KBError):
        kb.reduce_noalloc([x] * 7)                 # more than six arrays
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    import ctypes as C
    ptrs = (C.c_void_p * 1)(x.data_ptr())
    rc = kb.lib().kb_reduce_noalloc(ptrs, 1, (1 << 40) + 1, 0, C.c_void_p(out.data_ptr()), None)
    assert rc == kb.EINVAL

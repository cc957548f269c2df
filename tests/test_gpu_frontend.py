"""GPU tests of the automatic batching front-end (frontend.BatchedLoop):
user step functions of PyTorch-ROCm element-wise ops, run per launch and in
captured iteration batches.  Every replayed result is compared with the
eager result bit for bit (the graph replays the same kernels on the same
memory), over several calls with eager work and synchronisation between
them."""
import numpy as np
import pytest

from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    need_gpu()
    import torch
    return torch


def skeleton_state(torch, seed=5, n=1 << 16):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = (torch.rand(n, generator=g) * 2 - 1).cuda()
    a = [0.9 + 0.1 * float(v) for v in torch.rand(4, generator=g)]
    b = [0.02 * float(v) - 0.01 for v in torch.rand(4, generator=g)]
    return x, a, b


def make_step(x, a, b):
    def step():
        for k in range(4):
            x.mul_(a[k]).add_(b[k])
    return step


def test_batched_equals_eager_every_replay(torch):
    from paper_2501_09398_amd import frontend
    announce("frontend skeleton chain")
    x_e, a, b = skeleton_state(torch)
    x_g = x_e.clone()
    eager = frontend.batch(make_step(x_e, a, b))
    batched = frontend.batch(make_step(x_g, a, b))
    for call, (n, bb) in enumerate([(100, 7), (50, 7), (13, 7), (64, 8), (3, 7)]):
        eager.run(n, 0)
        r = batched.run(n, bb)
        torch.cuda.synchronize()
        assert torch.equal(x_e, x_g), call
        assert r["graph_launches"] == n // bb and r["peeled"] == n % bb
        x_e.add_(0.0)                       # eager work between the calls
        x_g.add_(0.0)
    assert set(batched._graphs) == {7, 8}


def test_alternating_buffers_with_even_batches(torch):
    """A step that writes the other buffer and swaps Python references:
    even batches restore the reference state after each replay."""
    from paper_2501_09398_amd import frontend
    announce("frontend ping-pong")
    g = torch.Generator(device="cpu").manual_seed(3)
    init = torch.rand(256, 256, generator=g).cuda() + 323.0

    def make(bufs):
        def step():
            src, dst = bufs[0], bufs[1]
            dst.copy_(src)
            dst[1:-1, 1:-1].add_(1e-3 * (src[:-2, 1:-1] + src[2:, 1:-1] + src[1:-1, :-2] + src[1:-1, 2:]
                                         - 4 * src[1:-1, 1:-1]))
            bufs.reverse()
        return step
    be = [init.clone(), torch.empty_like(init)]
    bg = [init.clone(), torch.empty_like(init)]
    eager, batched = frontend.batch(make(be)), frontend.batch(make(bg), state=bg)
    for n in (40, 40, 22):
        eager.run(n, 0)
        batched.run(n, 10)
        torch.cuda.synchronize()
        assert torch.equal(be[0], bg[0])
    # an odd b cannot be replayed (the buffers move over the recorded
    # calls): refused, the buffer list left as it was, and the state intact
    order = [t.data_ptr() for t in bg]
    with pytest.raises(ValueError):
        batched.run(21, 7)
    assert [t.data_ptr() for t in bg] == order
    eager.run(6, 0)
    batched.run(6, 2)
    torch.cuda.synchronize()
    assert torch.equal(be[0], bg[0])


def test_skeleton_step_against_float64_oracle(torch):
    """The front-end's skeleton step (torch element-wise multiply, then
    add: two roundings per kernel) from the seeded workload inputs, in
    graph batches, against the float64 oracle of the chain: within the
    round-off bound of the affine recurrence, 2K u max(|x|+|b|) per
    iteration, damped by the contraction A = a_4 a_3 a_2 a_1 < 1 (at most
    1/(1-A) iterations' worth accumulates)."""
    import oracle
    import synth
    from paper_2501_09398_amd import frontend
    announce("frontend skeleton vs float64 oracle")
    n, iters = 1 << 16, 300
    x0, a, b = synth.skeleton_init(20250116, n, 4)
    x = torch.from_numpy(x0.copy()).cuda()
    loop = frontend.batch(make_step(x, [float(v) for v in a], [float(v) for v in b]))
    loop.run(iters, 50)
    torch.cuda.synchronize()
    got = x.cpu().numpy().astype(np.float64)
    ref = oracle.skeleton(x0, a, b, iters)
    A = float(np.prod(a.astype(np.float64)))
    u = 2.0 ** -24
    bound = min(iters, 1.0 / (1.0 - A)) * 2 * 4 * u * (max(np.abs(ref).max(), np.abs(x0).max()) + np.abs(b).max())
    err = float(np.max(np.abs(got - ref)))
    print(f"frontend skeleton vs float64: max |err| {err:.3e} (bound {bound:.3e}), "
          f"vs the library's fused chain (float32 oracle) {np.max(np.abs(got - oracle.skeleton(x0, a, b, iters, dtype=np.float32))):.3e}")
    assert err <= bound


def test_tune_picks_an_admissible_batch(torch):
    from paper_2501_09398_amd import frontend
    announce("frontend tune")
    x, a, b = skeleton_state(torch, n=1 << 12)
    loop = frontend.batch(make_step(x, a, b))
    cands = [1, 2, 5, 10, 20, 50, 100, 200]
    res = loop.tune(1000, candidates=cands, probe_iters=200, reps=2)
    print({k: res[k] for k in ("b", "b_measured", "b_closed_form")})
    assert res["b"] in cands and res["b_measured"] in cands
    assert np.isfinite(res["model"]["creation"]["k_c"]) and res["model"]["creation"]["k_c"] > 0
    # graphs beat per-launch at the chosen b for this launch-bound loop
    x_ref = x.clone()
    t_g = loop.run(1000, res["b"])["t_exec_s"]
    ref = frontend.batch(make_step(x_ref, a, b))
    t_e = ref.run(1000, 0)["t_exec_s"]
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    print(f"per launch {t_e * 1e3:.2f} ms, batched b={res['b']} {t_g * 1e3:.2f} ms")
    assert t_g < t_e


"""Graph batching against the per-launch loop over seeded random
configurations: problem, shape, kernel variant, temporal depth, builder,
batch size b and a split of the steps over several kb_run calls.  The
graph arm must give the per-launch arm's bits in every case (the paper's
graphs replay the same kernels on the same memory; here that includes the
parity graphs of the alternating buffers, loop peeling, the steps left
over by temporal blocking, and the FDTD step counter)."""
import numpy as np
import pytest

from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

HEAT = (1e-3, 1.0, 1.0, 10.0, 300.0)


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def configs():
    rng = np.random.default_rng(20250116)
    out = []
    for case in range(24):
        kind = ("HEAT2D", "HEAT3D", "SKELETON", "FDTD3D", "HEAT2D_MULTI")[case % 5]
        if kind == "HEAT2D":
            shape = (int(rng.integers(1, 90)), int(rng.integers(1, 90)) * 4)
            variant = int(rng.choice([1, 2, 5, 6, 9, 13, 15, 16, 17, 18, 19, 20, 21, 22, 23]))
            depth = int(rng.integers(1, 9)) if variant in (2, 5, 6, 15, 16, 17, 18, 19, 20, 21, 22, 23) else 1
        elif kind == "HEAT3D":
            shape = (int(rng.integers(1, 9)), int(rng.integers(1, 50)), int(rng.integers(1, 30)) * 4)
            variant = int(rng.choice([1, 2, 5, 6, 11]))
            depth = int(rng.integers(1, 7)) if variant in (5, 11) else 1
        elif kind == "SKELETON":
            shape = (int(rng.integers(1, 5000)),)
            variant, depth = int(rng.choice([1, 2, 3])), 1
        elif kind == "FDTD3D":
            shape = (int(rng.integers(4, 20)), 512)
            variant, depth = int(rng.choice([1, 2, 3, 5, 6, 7])), 1
        else:
            g = int(rng.integers(1, 5))
            sides = [int(s) for s in rng.integers(1, 140, size=2 * g)]
            shape = [g] + sides
            variant = int(rng.choice([1, 2, 3, 4, 5, 6]))
            depth = int(rng.integers(1, 9)) if variant in (3, 4, 5, 6) else 1
        b = int(rng.integers(1, 12))
        builder = int(rng.integers(0, 2))
        runs = [int(r) for r in rng.integers(0, 40, size=int(rng.integers(1, 4)))]
        out.append((kind, tuple(shape), variant, depth, b, builder, tuple(runs)))
    return out


def coeffs_for(kb, kind):
    return {"HEAT2D": HEAT, "HEAT3D": HEAT, "HEAT2D_MULTI": HEAT, "SKELETON": (4,),
            "FDTD3D": kb.FDTD_COEFFS}[kind]


def state(kb, p, kind):
    if kind == "SKELETON":
        return [p.read(kb.F_X)]
    if kind == "FDTD3D":
        return [p.read(fid) for fid in kb.FDTD_FIELDS.values()] + [p.read(kb.F_PROBE), p.read(kb.F_STEP)]
    return [p.read(kb.F_T)]


@pytest.mark.parametrize("cfg", configs(), ids=lambda c: f"{c[0]}-{c[1]}-v{c[2]}-t{c[3]}-b{c[4]}-B{c[5]}")
def test_graph_batches_equal_per_launch(kb, cfg):
    kind, shape, variant, depth, b, builder, runs = cfg
    announce(f"graph fuzz {cfg}")
    outs = []
    for bb in (0, b):
        with kb.Problem(getattr(kb, kind), shape, coeffs_for(kb, kind), 7) as p:
            p.set_option(kb.OPT_TILE, variant)
            p.set_option(kb.OPT_TDEPTH, depth)
            p.set_option(kb.OPT_BUILDER, builder)
            for n in runs:
                p.run(n, bb)
            outs.append(state(kb, p, kind))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)

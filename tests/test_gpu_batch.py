"""Batched persistent solves (one launch, many uneven systems) through the C
ABI: every system's result equals its own single mixed-precision solve bit
for bit when the batch uses the single solve's row partition, stays within
the refinement tolerance of the FP64 oracle, and the scheduler always
drains (including when the host forces its stall guard)."""
import numpy as np
import pytest

import oracle
from paper_2501_03743_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2501_03743_amd import sstep
    with sstep.Handle(0) as h:
        yield h


def _systems(H, sides, seed0=0, sigma=0.5):
    mats, ks, bs, keep = [], [], [], []
    for i, L in enumerate(sides):
        shape = (int(L), int(L), int(L))
        k = np.exp(wl.gaussian_random_field(shape, sigma, 0.1, seed0 + i))
        kd = torch.from_numpy(k).cuda()
        mats.append(H.matrix_stencil("3d7_vark", shape, k=kd))
        ks.append(k)
        bs.append(torch.from_numpy(wl.normal_rhs(L ** 3, seed0 + i)).cuda())
        keep.append(kd)
    return mats, ks, bs, keep


def test_batch_equals_single_solves_bitwise(H):
    sides = [12, 20, 7, 33, 16, 41, 9, 24]
    mats, ks, bs, keep = _systems(H, sides)
    xs = [torch.zeros_like(b) for b in bs]
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=4, rtol=1e-8)
    assert rc == 0 and (st == 0).all(), st
    for i, (M, b) in enumerate(zip(mats, bs)):
        x1 = torch.zeros_like(b)
        r = H.solve(M, b, x1, s=4, rtol=1e-8, precision="mixed_ir")
        assert r.status == 0
        assert torch.equal(x1, xs[i]), (i, sides[i])
        assert r.outer == it[i], (i, r.outer, it[i])
        assert tr[i] <= 1e-8 and abs(tr[i] - r.true_rel) <= 1e-12 * max(tr[i], 1e-300) + 1e-20
    for M in mats:
        M.close()


def test_batch_skewed_sizes_against_oracle(H):
    sides = [32, 64, 40, 96, 48, 36, 80, 32]
    mats, ks, bs, keep = _systems(H, sides, seed0=100)
    xs = [torch.zeros_like(b) for b in bs]
    from paper_2501_03743_amd import sstep
    tune = sstep.Tune(tile_rows=16384, grid=512, order=0)
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=4, rtol=1e-8, tune=tune)
    assert rc == 0 and (st == 0).all(), st
    assert (tr <= 1e-8).all()
    for i in (0, 2, 7):
        shape = (sides[i],) * 3
        ref = oracle.sstep(oracle.Operator("3d7_vark", shape, k=ks[i]), bs[i].cpu().numpy(), 4,
                           rtol=1e-12, maxit=50000)
        xg = xs[i].cpu().numpy()
        err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
        print("batch system %d (L=%d): inner iterations %d, err vs oracle %.2e, true rel %.2e"
              % (i, sides[i], it[i], err, tr[i]))
        assert err <= 1e-5
    for M in mats:
        M.close()


def test_batch_round_robin_and_mixed_edge_cases(H):
    from paper_2501_03743_amd import sstep
    sides = [10, 30, 8]
    mats, ks, bs, keep = _systems(H, sides, seed0=200)
    bs[1] = torch.zeros_like(bs[1])      # zero right-hand side
    xs = [torch.ones_like(b) for b in bs]
    tune = sstep.Tune(tile_rows=4096, grid=64, order=1)
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=3, rtol=1e-9, tune=tune)
    assert rc == 0 and (st == 0).all(), st
    assert not xs[1].cpu().numpy().any()
    assert tr[0] <= 1e-9 and tr[2] <= 1e-9
    xs = [torch.zeros_like(b) for b in bs]
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=3, rtol=1e-14, max_refine=1)
    assert rc == sstep.NOT_CONVERGED and st[0] == sstep.NOT_CONVERGED and st[1] == 0
    with pytest.raises(sstep.SspError):
        H.solve_batch(mats, bs, xs, s=9)
    for M in mats:
        M.close()


def test_batch_stall_guard_forced_from_host(H):
    """A spin limit of one poll makes idle workgroups give up almost at once:
    the launch must still end and the call must report the stall."""
    from paper_2501_03743_amd import sstep
    sides = [40, 40, 40, 40]
    mats, ks, bs, keep = _systems(H, sides, seed0=300)
    xs = [torch.zeros_like(b) for b in bs]
    tune = sstep.Tune(tile_rows=65536, grid=1024, order=1, spin_limit=1)
    try:
        H.solve_batch(mats, bs, xs, s=4, rtol=1e-8, tune=tune)
        finished = True
    except sstep.SspError as e:
        assert e.code == sstep.EHIP and "stalled" in str(e)
        finished = False
    # either way the device is usable afterwards
    xs = [torch.zeros_like(b) for b in bs]
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=4, rtol=1e-8)
    assert rc == 0
    print("stall guard triggered:", not finished)
    for M in mats:
        M.close()


def test_autotune_and_cache(H, tmp_path):
    sides = [24, 16, 32, 20]
    mats, ks, bs, keep = _systems(H, sides, seed0=400)
    cache = str(tmp_path / "tune.txt")
    t1 = H.autotune_batch(mats, bs, s=4, cache_path=cache)
    assert t1.grid > 0 or t1.schedule == 1
    text = open(cache).read()
    assert "gfx950" in text and "schedule=%d" % t1.schedule in text
    t2 = H.autotune_batch(mats, bs, s=4, cache_path=cache)
    assert t2.as_dict() == t1.as_dict()
    xs = [torch.zeros_like(b) for b in bs]
    rc, st, it, tr = H.solve_batch(mats, bs, xs, s=4, rtol=1e-8, tune=t1)
    assert rc == 0
    for M in mats:
        M.close()


@pytest.mark.parametrize("tile_rows", [0, 4096])
def test_stepped_schedule_equals_persistent_bitwise(H, tile_rows):
    """The stepped schedule (one launch pair per phase step) and the
    persistent kernel claiming one tile or runs of 3 or 8 tiles at a time run
    each tile's arithmetic identically: same results bit for bit, for uneven
    systems that finish at different steps."""
    from paper_2501_03743_amd import sstep
    sides = [28, 9, 45, 17, 33, 6]
    mats, ks, bs, keep = _systems(H, sides, seed0=500)
    out = {}
    for sched, run in ((0, 1), (1, 0), (0, 3), (0, 8)):
        xs = [torch.zeros_like(b) for b in bs]
        tune = sstep.Tune(tile_rows=tile_rows, grid=256, order=0, schedule=sched, run=run)
        rc, st, it, tr = H.solve_batch(mats, bs, xs, s=4, rtol=1e-9, tune=tune)
        assert rc == 0 and (st == 0).all(), (sched, run, st)
        out[(sched, run)] = (xs, it.copy(), tr.copy())
    for key in ((0, 1), (0, 3), (0, 8)):
        for i in range(len(sides)):
            assert torch.equal(out[key][0][i], out[(1, 0)][0][i]), (key, i)
        assert (out[key][1] == out[(1, 0)][1]).all(), key
        assert np.array_equal(out[key][2], out[(1, 0)][2]), key
    out[1] = out[(1, 0)]
    if tile_rows == 0:
        for i, (M, b) in enumerate(zip(mats, bs)):
            x1 = torch.zeros_like(b)
            r = H.solve(M, b, x1, s=4, rtol=1e-9, precision="mixed_ir")
            assert torch.equal(x1, out[1][0][i]), i
    for M in mats:
        M.close()

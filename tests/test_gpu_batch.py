"""GPU checks of the batched form: uneven volumes with their own PSFs, one
graph launch per iteration, against the FP64 oracle and against single-volume
plans (same kernels, so equal bit for bit)."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14143_amd import rl, synth

pytestmark = pytest.mark.gpu

SHAPES = [(12, 24, 24), (16, 32, 32), (12, 24, 24), (24, 48, 48), (16, 32, 32), (8, 16, 64)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def cases():
    out = []
    for i, shp in enumerate(SHAPES):
        sig = (1.0 + 0.3 * i, 1.2 + 0.2 * i, 2.0 + 0.25 * i)
        out.append(synth.small_case(shp, sigma_xyz=sig, seed=20 + i, density=4.0))
    return out


def test_batch_matches_oracle_and_single_plans(torch):
    say("batch vs oracle and single plans")
    cs = cases()
    n_iter = 10
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs]) as bp:
        d = [dev(torch, c["d"]) for c in cs]
        u = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, u, n_iter)
        flux = bp.flux()
    assert flux.shape == (len(cs), n_iter)
    for i, c in enumerate(cs):
        ref, ref_flux, _ = oracle.rl(c["d"], c["psf"], c["u0"], n_iter)
        got = u[i].cpu().numpy()
        err = oracle.rel_l2(got, ref)
        say("  volume", i, c["shape"], "relL2", err)
        assert err <= 1e-4
        assert np.max(np.abs(flux[i] - ref_flux) / ref_flux) <= 1e-6
        with rl.Plan(dev(torch, c["psf"])) as p:
            us = dev(torch, c["u0"])
            p.iterate(d[i], us, n_iter)
            torch.cuda.synchronize()
        assert torch.equal(us, u[i]), i


@pytest.fixture(scope="module")
def batch96():
    return synth.make_batch(96)


@pytest.mark.parametrize("autotune", [True, False])
def test_full_size_batch_workload(torch, batch96, autotune):
    # the benchmark's batch: 96 uneven volumes (about 1e8 voxels, five shape
    # classes) in one plan as it is timed (autotuned; the default shapes too); the
    # first volume of every class element by element against the oracle, and every
    # volume's flux against its data
    vols = batch96
    n_iter = 2
    say("full-size batch", len(vols), "volumes, autotune", autotune)
    first = {}
    for i, v in enumerate(vols):
        first.setdefault(tuple(v["shape"]), i)
    with rl.BatchPlan([dev(torch, v["psf"]) for v in vols], autotune=autotune) as bp:
        d = [dev(torch, v["d"]) for v in vols]
        u = [dev(torch, v["u0"]) for v in vols]
        bp.iterate(d, u, n_iter)
        flux = bp.flux()
        got = {i: u[i].cpu().numpy() for i in first.values()}
    assert flux.shape == (len(vols), n_iter)
    for i, v in enumerate(vols):
        total = float(v["d"].sum(dtype=np.float64))
        assert np.all(np.abs(flux[i] - total) / total <= 1e-6), (i, flux[i], total)
    for shp, i in first.items():
        ref = oracle.rl(vols[i]["d"], vols[i]["psf"], vols[i]["u0"], n_iter)[0]
        err = oracle.rel_l2(got[i], ref)
        say("  class", shp, "volume", i, "relL2", err)
        assert err <= 1e-5


def test_batch_graph_replays_and_resume(torch):
    say("batch graph replays")
    cs = cases()
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs]) as bp:
        d = [dev(torch, c["d"]) for c in cs]
        a = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, a, 7)
        b = [dev(torch, c["u0"]) for c in cs]
        for k in (3, 1, 3):  # separate calls replay the same graphs
            bp.iterate(d, b, k)
            junk = torch.randn(1 << 20, device="cuda:0")  # eager work between replays
            junk.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        for i in range(len(cs)):
            assert torch.equal(a[i], b[i]), i
        # one iteration, then zero (no-op)
        e = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, e, 1)
        bp.iterate(d, e, 0)
        torch.cuda.synchronize()
        assert bp.flux().shape == (len(cs), 1)


def test_batch_more_iterations_than_initial_capacity(torch):
    # 130 > initial flux capacity: partial tables grow and the graphs are rebuilt
    say("batch capacity growth")
    cs = cases()[:2]
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs]) as bp:
        d = [dev(torch, c["d"]) for c in cs]
        u = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, u, 3)
        bp.iterate(d, u, 130)
        f = bp.flux()
    assert f.shape == (2, 130)
    for i, c in enumerate(cs):
        total = float(c["d"].sum(dtype=np.float64))
        assert np.all(np.abs(f[i] - total) / total <= 1e-6)


def test_batch_errors(torch):
    say("batch errors")
    cs = cases()[:2]
    psfs = [dev(torch, c["psf"]) for c in cs]
    with pytest.raises(rl.RLError):
        rl.rl_plan_create_batch([], [])
    bad = cs[0]["psf"].copy()
    bad[0, 0, 0] = -1
    with pytest.raises(rl.RLError) as ei:
        rl.BatchPlan([psfs[0], dev(torch, bad)])
    assert ei.value.status == rl.RL_E_INVALID
    with rl.BatchPlan(psfs) as bp:
        d = [dev(torch, c["d"]) for c in cs]
        u = [dev(torch, c["u0"]) for c in cs]
        host = np.ones(16, np.float32)
        with pytest.raises(rl.RLError) as ei:  # a host pointer is refused
            rl.rl_iterate_batch(bp.handle, [d[0].data_ptr(), host.ctypes.data],
                                [u[0].data_ptr(), u[1].data_ptr()], 1)
        assert ei.value.status == rl.RL_E_INVALID
        with pytest.raises(rl.RLError):
            rl.rl_iterate_batch(bp.handle, [d[0].data_ptr(), d[1].data_ptr()],
                                [u[0].data_ptr(), u[1].data_ptr()], -1)
        with pytest.raises(rl.RLError):
            rl.rl_iterate(bp.handle, d[0].data_ptr(), u[0].data_ptr(), 1)
        with pytest.raises(rl.RLError):
            rl.conv3d_fft(bp.handle, d[0].data_ptr(), u[0].data_ptr())


BATCH_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                            "rl_batch96_samples.txt")


def batch_golden():
    """{volume: (points, values)} and {volume: flux} of the FP64 oracle after 50
    iterations, written by tests/golden/make_rl_batch96_samples.py (oracle only)."""
    flux, pts = {}, {}
    with open(BATCH_GOLDEN) as f:
        for line in f:
            if line.startswith("# flux "):
                _, _, v, val = line.split()
                flux[int(v)] = float(val)
    a = np.loadtxt(BATCH_GOLDEN, comments="#")
    for v in np.unique(a[:, 0]).astype(int):
        rows = a[a[:, 0] == v]
        pts[v] = (rows[:, 1:4].astype(np.int64), rows[:, 4])
    return pts, flux


def test_full_size_batch_workload_50_iterations(torch, batch96):
    # the benchmark's batch as it is timed (autotuned, 50 iterations, graph replays):
    # the first and last volume of every shape class against the oracle's stored
    # estimate at sampled voxels, every volume's flux against its data, and the
    # stored volumes' flux against the oracle's
    vols = batch96
    n_iter = 50
    pts, ref_flux = batch_golden()
    shapes = {tuple(vols[v]["shape"]) for v in pts}
    assert len(shapes) == 5 and len(pts) == 10  # two volumes of every class
    say("full-size batch, 50 iterations, volumes", sorted(pts))
    with rl.BatchPlan([dev(torch, v["psf"]) for v in vols], autotune=True) as bp:
        d = [dev(torch, v["d"]) for v in vols]
        u = [dev(torch, v["u0"]) for v in vols]
        bp.iterate(d, u, n_iter)
        flux = bp.flux()
        got = {v: u[v].cpu().numpy().astype(np.float64) for v in pts}
    for i, v in enumerate(vols):
        total = float(v["d"].sum(dtype=np.float64))
        assert np.all(np.abs(flux[i] - total) / total <= 1e-6), (i, flux[i][-1], total)
    for v, (p, ref) in sorted(pts.items()):
        g = got[v][tuple(p.T)]
        err = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
        worst = float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
        say("  volume", v, vols[v]["shape"], "relL2 over", len(ref), "samples", err,
            "max abs / peak", worst)
        assert err <= 1e-4
        assert abs(flux[v][-1] - ref_flux[v]) / ref_flux[v] <= 1e-6


# shapes whose every pass splits into the persistent kernel's 128-thread work-groups;
# their launch shapes hold the same elements per thread on Y and Z (ny = 2 nz)
PERSIST_SHAPES = [(24, 48, 48), (32, 64, 64), (24, 48, 48), (48, 96, 96), (32, 64, 64)]
PERSIST_ELEMS = {(24, 48, 48): (6, 6), (32, 64, 64): (4, 8), (48, 96, 96): (6, 12)}


# The library refuses the persistent mode: a run of the first test below did not
# finish within its two-minute limit, and neither did the one that tested a change
# of its completion polls (which, as it turned out, the compiler had folded back
# into the same plain loads).  Its tests stay, skipped, until the mode is switched
# on again.
PERSIST_OFF = pytest.mark.skip(reason="persistent batched kernel switched off: its completion "
                                      "waits did not finish on the GPU")


def persist_cases():
    out = []
    for i, shp in enumerate(PERSIST_SHAPES):
        sig = (1.0 + 0.3 * i, 1.2 + 0.2 * i, 2.0 + 0.25 * i)
        out.append(synth.small_case(shp, sigma_xyz=sig, seed=40 + i, density=2.0))
    return out


@PERSIST_OFF
def test_persistent_batch_matches_oracle_and_single_plans(torch):
    # one persistent launch per iteration: every volume against the oracle, and bit
    # for bit against single-volume plans with the same elements per thread (the
    # same kernels' arithmetic, run as persistent tiles)
    say("persistent batch vs oracle and single plans")
    cs = persist_cases()
    n_iter = 10
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs], mode="persistent") as bp:
        assert bp.mode() == "persistent"
        d = [dev(torch, c["d"]) for c in cs]
        u = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, u, n_iter)
        flux = bp.flux()
    for i, c in enumerate(cs):
        ref, ref_flux, _ = oracle.rl(c["d"], c["psf"], c["u0"], n_iter)
        got = u[i].cpu().numpy()
        err = oracle.rel_l2(got, ref)
        say("  volume", i, c["shape"], "relL2", err)
        assert err <= 1e-4
        assert np.max(np.abs(flux[i] - ref_flux) / ref_flux) <= 1e-6
        xe, yze = PERSIST_ELEMS[tuple(c["shape"])]
        with rl.Plan(dev(torch, c["psf"]), x_elems=xe, yz_elems=yze) as p:
            us = dev(torch, c["u0"])
            p.iterate(d[i], us, n_iter)
            fs = p.flux()
        assert torch.equal(us, u[i]), i
        assert np.array_equal(fs, flux[i]), i


@PERSIST_OFF
def test_persistent_batch_replays_resume_and_growth(torch):
    # separate calls replay the same two graphs (one persistent launch each); a call
    # longer than the counters' and partials' capacity grows them and re-captures
    say("persistent batch replays")
    cs = persist_cases()
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs], mode="persistent") as bp:
        d = [dev(torch, c["d"]) for c in cs]
        a = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, a, 7)
        b = [dev(torch, c["u0"]) for c in cs]
        for k in (3, 1, 3):
            bp.iterate(d, b, k)
            junk = torch.randn(1 << 20, device="cuda:0")  # eager work between replays
            junk.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        for i in range(len(cs)):
            assert torch.equal(a[i], b[i]), i
        g = [dev(torch, c["u0"]) for c in cs]
        bp.iterate(d, g, 130)
        f = bp.flux()
    assert f.shape == (len(cs), 130)
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cs], mode="graph") as gp:
        assert gp.mode() == "graph"
        h = [dev(torch, c["u0"]) for c in cs]
        gp.iterate(d, h, 130)
    for i, c in enumerate(cs):
        total = float(c["d"].sum(dtype=np.float64))
        assert np.all(np.abs(f[i] - total) / total <= 1e-6), i
        # the graph form (its own launch shapes) agrees to rounding
        err = float(torch.linalg.vector_norm((g[i] - h[i]).double()) /
                    torch.linalg.vector_norm(h[i].double()))
        assert err <= 1e-5, (i, err)


def test_persistent_mode_refused(torch):
    # the switched-off persistent mode is refused with RL_E_UNSUPPORTED, also for
    # shapes its launch shapes would fit; "auto" runs the per-pass graph
    for cs in (cases(), persist_cases()):
        psfs = [dev(torch, c["psf"]) for c in cs]
        with pytest.raises(rl.RLError) as ei:
            rl.BatchPlan(psfs, mode="persistent")
        assert ei.value.status == rl.RL_E_UNSUPPORTED
        with rl.BatchPlan(psfs) as bp:
            assert bp.mode() == "graph"
            assert not bp.launch()["batch_persistent"]


@PERSIST_OFF
def test_benchmark_batch_runs_persistent(torch, batch96):
    # every shape class of the benchmark's batch fits the persistent kernel
    with rl.BatchPlan([dev(torch, v["psf"]) for v in batch96[:12]]) as bp:
        assert bp.mode() == "persistent"

"""Batched form: instances advanced together must follow exactly the
single-instance solver (same kernels, same cycle sequence), and one of them
the CPU oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import cfas
from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def small_ensemble():
    out = []
    for i, n in enumerate([8, 12, 16, 24, 32, 48, 6, 32]):
        g = inputs.rng(4000 + i)
        eps = float(g.uniform(0.02, 0.3))
        mean = float(g.uniform(0.05, 0.3))
        L = n * math.pi / 4
        phi0 = mean + 0.05 * g.uniform(-1, 1, (n, n, n))
        out.append(dict(n=n, L=L, eps=eps, dt=0.1, phi0=phi0))
    return out


@pytest.mark.parametrize("cycle,nu", [("V", (2, 2)), ("F", (2, 2)), ("V", (0, 2)), ("V", (1, 1))])
def test_batch_matches_single_instances(cycle, nu):
    from paper_1611_06288_amd.solver import Batch, Solver
    ens = small_ensemble()
    steps = 3
    b = Batch(ens, tol=1e-10, cycle=cycle, nu1=nu[0], nu2=nu[1])
    for i, p in enumerate(ens):
        b.init_state(i, dev(p["phi0"]))
    infos = b.run(steps)
    for i, p in enumerate(ens):
        s = Solver(p["n"], p["L"], p["eps"], p["dt"], tol=1e-10, cycle=cycle, nu1=nu[0],
                   nu2=nu[1])
        prev, cur, mu, om, sinfos = s.simulate(dev(p["phi0"]), steps)
        bprev, bcur, bmu, bom = b.get_state(i)
        assert [x.cycles for x in infos[i]] == [x.cycles for x in sinfos], i
        err = float((bcur - cur).abs().max() / cur.abs().max())
        assert err <= 1e-13, (i, err)
        assert float((bprev - prev).abs().max()) <= 1e-13 * float(prev.abs().max())
        assert float((bmu - mu).abs().max()) <= 1e-12 * float(mu.abs().max())


def test_batch_instance_matches_oracle_and_autotune_keeps_results(tmp_path):
    from paper_1611_06288_amd.solver import Batch
    ens = small_ensemble()[:5]
    steps = 2
    b = Batch(ens, tol=1e-10)                          # default tile shapes
    b2 = Batch(ens, tol=1e-10)
    tiles = b2.autotune(cache_path=tmp_path / "tiles.json")
    assert len(tiles) == 5
    assert all(th in (64, 128, 256) and w in (64, 128, 256, 512, 1024) and w >= th
               and z in (1, 2, 4, 8) for _, th, w, z in tiles)
    assert (tmp_path / "tiles.json").exists()
    b3 = Batch(ens, tol=1e-10)
    assert b3.autotune(cache_path=tmp_path / "tiles.json") == tiles   # read back from the cache
    b3.close()
    for bb in (b, b2):
        for i, p in enumerate(ens):
            bb.init_state(i, dev(p["phi0"]))
    i1 = b.run(steps)
    i2 = b2.run(steps)          # per-point arithmetic does not depend on the tiles
    for i, p in enumerate(ens):
        assert [x.cycles for x in i1[i]] == [x.cycles for x in i2[i]]
        assert torch.equal(b.get_state(i)[1], b2.get_state(i)[1])
    # instance 3 (24^3) against the oracle
    p = ens[3]
    phis, oinfos, _ = cfas.simulate(p["phi0"], p["L"], p["eps"], p["dt"], steps, tol=1e-10)
    got = b.get_state(3)[1].cpu().numpy()
    assert [x.cycles for x in i1[3]] == [x.cycles for x in oinfos]
    assert np.max(np.abs(got - phis[-1])) / np.max(np.abs(phis[-1])) < 1e-11


def test_batch_64_instances_uneven():
    """The 64-instance ensemble (n in {32,48,64,96}, eps in [0.02,0.3]) for two
    steps; four instances, one of each size, against single-instance runs."""
    from paper_1611_06288_amd.solver import Batch, Solver
    ens = inputs.batched_ensemble(64, steps=2)
    params = [dict(n=e.params.n, L=e.params.L, eps=e.params.eps, dt=e.params.dt) for e in ens]
    b = Batch(params, tol=1e-10)
    for i, e in enumerate(ens):
        b.init_state(i, dev(e.phi0()))
    infos = b.run(2)
    assert all(x.status == 0 and x.res_final <= 1e-10 for row in infos for x in row)
    seen = set()
    for i, e in enumerate(ens):
        if e.params.n in seen:
            continue
        seen.add(e.params.n)
        p = e.params
        s = Solver(p.n, p.L, p.eps, p.dt, tol=1e-10)
        _, cur, _, _, sinfos = s.simulate(dev(e.phi0()), 2)
        assert [x.cycles for x in infos[i]] == [x.cycles for x in sinfos]
        assert float((b.get_state(i)[1] - cur).abs().max()) <= 1e-13 * float(cur.abs().max())
    assert seen == {32, 48, 64, 96}


def test_batch_statuses_per_instance():
    """Per-instance stop tests: with max_cycles = 2 and an unreachable tol
    every instance ends NOT_CONVERGED after exactly 2 cycles with the
    single-instance solver's residuals; an instance whose state holds a NaN
    ends NONFINITE while the others converge as they do alone."""
    from paper_1611_06288_amd.solver import Batch, Solver
    ens = small_ensemble()[:4]
    b = Batch(ens, tol=1e-14, max_cycles=2)
    for i, p in enumerate(ens):
        b.init_state(i, dev(p["phi0"]))
    infos = b.run(1, raise_on_error=False)
    for i, p in enumerate(ens):
        x = infos[i][0]
        assert (x.status, x.cycles) == (2, 2), (i, x)
        s = Solver(p["n"], p["L"], p["eps"], p["dt"], tol=1e-14, max_cycles=2)
        phi = dev(p["phi0"])
        mu, om = s.init_guess(phi)
        _, y = s.step(phi, phi, mu, om, raise_on_error=False)
        assert y.status == 2 and y.cycles == 2
        assert x.res0 == pytest.approx(y.res0, rel=1e-12)
        assert x.res_final == pytest.approx(y.res_final, rel=1e-9)
    b2 = Batch(ens, tol=1e-10)
    for i, p in enumerate(ens):
        phi = dev(p["phi0"])
        if i == 1:
            phi[1, 2, 3] = float("nan")
        b2.init_state(i, phi)
    infos = b2.run(1, raise_on_error=False)
    assert infos[1][0].status == 3
    for i, p in enumerate(ens):
        if i == 1:
            continue
        s = Solver(p["n"], p["L"], p["eps"], p["dt"], tol=1e-10)
        _, _, _, _, sinfos = s.simulate(dev(p["phi0"]), 1)
        assert infos[i][0].status == 0 and infos[i][0].cycles == sinfos[0].cycles, i


def test_batch_column_tiled_interpolation_is_bitwise_the_two_pass_form():
    """When every instance's finest size is a multiple of 16 the finest
    interpolation runs as column tiles that form the coarse error themselves;
    adding one instance of another size (24) sends the whole finest depth
    through the coarse-error pass and the per-pair interpolation instead.
    The instances the two batches share must come out bit for bit equal."""
    from paper_1611_06288_amd.solver import Batch
    shared = []
    for i, n in enumerate([16, 32, 48, 32]):
        g = inputs.rng(5100 + i)
        shared.append(dict(n=n, L=n * math.pi / 4, eps=float(g.uniform(0.05, 0.3)), dt=0.1,
                           phi0=0.2 + 0.05 * g.uniform(-1, 1, (n, n, n))))
    extra = dict(n=24, L=6 * math.pi, eps=0.2, dt=0.1,
                 phi0=0.2 + 0.05 * inputs.rng(5199).uniform(-1, 1, (24, 24, 24)))
    results = []
    for ens in (shared, shared + [extra]):
        b = Batch(ens, tol=1e-10)
        for i, p in enumerate(ens):
            b.init_state(i, dev(p["phi0"]))
        infos = b.run(2)
        results.append(([[x.cycles for x in row] for row in infos[:len(shared)]],
                        [b.get_state(i) for i in range(len(shared))]))
    (ca, sa), (cb, sb) = results
    assert ca == cb
    for i in range(len(shared)):
        for x, y in zip(sa[i], sb[i]):
            assert torch.equal(x, y), i


def test_batch_autotune_column_tiles_cached_and_bitwise(tmp_path):
    """On sizes that admit the column-tiled interpolation the autotuner also
    chooses between it and the two-pass form; the choice is cached (a second
    batch reads it back) and either choice gives the default batch's results
    bit for bit."""
    from paper_1611_06288_amd.solver import Batch
    ens = []
    for i, n in enumerate([16, 32, 48, 32]):
        g = inputs.rng(5300 + i)
        ens.append(dict(n=n, L=n * math.pi / 4, eps=float(g.uniform(0.05, 0.3)), dt=0.1,
                        phi0=0.2 + 0.05 * g.uniform(-1, 1, (n, n, n))))
    cache = tmp_path / "tiles.json"
    b = Batch(ens, tol=1e-10)
    b2 = Batch(ens, tol=1e-10)
    tiles = b2.autotune(cache_path=cache)
    text = cache.read_text()
    assert "prolong_tile" in text, text
    b3 = Batch(ens, tol=1e-10)
    assert b3.autotune(cache_path=cache) == tiles
    b3.close()
    _, th, w, z = tiles[3]
    print(f"interpolation choice: {tiles[3]}", flush=True)
    assert (th, w) == (64, 64) or z in (1, 2, 4, 8)
    for bb in (b, b2):
        for i, p in enumerate(ens):
            bb.init_state(i, dev(p["phi0"]))
    i1, i2 = b.run(2), b2.run(2)
    for i in range(len(ens)):
        assert [x.cycles for x in i1[i]] == [x.cycles for x in i2[i]]
        assert all(torch.equal(x, y) for x, y in zip(b.get_state(i), b2.get_state(i))), i

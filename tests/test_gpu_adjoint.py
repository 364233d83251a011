"""Adjoint step and differentiable rollout against references.

* one adjoint step against the implicit-function-theorem adjoint with dense
  matrices (8^3, definition oracle);
* a 3-step rollout gradient (phi0 and eps) against the dense-Jacobian
  rollout gradient of the definition oracle (8^3);
* the 64^3 adjoint workload (eps = 0.1, s = 0.1, 20 steps, checkpoints every
  5 steps): gradient along a seeded unit direction and d/deps against
  central finite differences (delta = 1e-6) of the same GPU forward map;
  bar 1e-6 relative.  A central difference at delta = 1e-6 resolves the map
  only as well as each forward solve: the solver's error divided by delta
  (residual 1e-13 -> ~1.6e-6 relative here, 1e-14 -> ~3.5e-7, while at
  delta = 1e-3 the two agree to 7e-10), so the forward runs to a residual
  of 1e-14, near the rounding floor of this grid."""
import math

import numpy as np
import pytest
import torch

from oracle import definition as D
from paper_1611_06288_amd import inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("n,cycle", [(8, "V"), (12, "F")])
def test_adjoint_step_matches_dense(n, cycle):
    from paper_1611_06288_amd import Solver
    L, eps, tau = n * 1.2, 0.2, 0.3
    h = L / n
    g = inputs.rng(50 + n)
    phk = 0.25 + 0.08 * g.uniform(-1, 1, (n, n, n))
    phkm1 = phk + 0.01 * g.uniform(-1, 1, (n, n, n))
    solver = D.solve_step_dense if n <= 8 else D.solve_step_nk
    u = solver(phkm1, phk, h, eps, tau)
    gbar = g.standard_normal((n, n, n))
    if n <= 8:
        ra, rb, re = D.adjoint_step_dense(phkm1, phk, u, gbar, h, eps, tau)
    s = Solver(n, L, eps, tau, cycle=cycle)
    gcur = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    gprev = torch.zeros_like(gcur)
    geps = torch.zeros(1, dtype=torch.float64, device="cuda")
    cyc = s.adjoint_step(dev(phkm1), dev(phk), dev(u[0]), dev(gbar), gcur, gprev, geps, adj_tol=1e-13)
    assert cyc > 0
    if n <= 8:
        assert rel(host(gcur), ra) < 1e-10
        assert rel(host(gprev), rb) < 1e-10
        assert float(geps[0]) == pytest.approx(re, rel=1e-10)
    # bootstrap aliasing: both contributions land in the same buffer
    gsum = torch.zeros_like(gcur)
    geps2 = torch.zeros_like(geps)
    s.adjoint_step(dev(phkm1), dev(phk), dev(u[0]), dev(gbar), gsum, gsum, geps2, adj_tol=1e-13)
    assert rel(host(gsum), host(gcur) + host(gprev)) < 1e-12
    # accumulation: a second call adds the same amounts again
    s.adjoint_step(dev(phkm1), dev(phk), dev(u[0]), dev(gbar), gcur, gprev, geps, adj_tol=1e-13)
    if n <= 8:
        assert rel(host(gcur), 2 * ra) < 1e-10


def test_rollout_gradient_matches_dense_8():
    from paper_1611_06288_amd.autograd import rollout
    n, L, eps, tau, steps = 8, 8.0, 0.15, 0.2, 3
    h = L / n
    phi0 = 0.2 + 0.05 * inputs.random_field(n, 61)
    target = 0.2 + 0.05 * inputs.random_field(n, 62)
    loss_ref, g_ref, ge_ref = D.rollout_loss_grad_dense(phi0, target, h, eps, tau, steps)
    p0 = dev(phi0).requires_grad_(True)
    e = torch.tensor(eps, dtype=torch.float64, requires_grad=True)
    params = dict(n=n, L=L, dt=tau, tol=1e-13, max_cycles=500, adj_tol=1e-13)
    out = rollout(p0, e, params, steps, ckpt_every=2)
    loss = ((out - dev(target)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(loss_ref, rel=1e-10)
    assert rel(host(p0.grad), g_ref) < 1e-9
    assert float(e.grad) == pytest.approx(ge_ref, rel=1e-9)


def test_adjoint_workload_64_finite_differences():
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.autograd import rollout
    p = inputs.adjoint_params(64)
    params = dict(n=p.n, L=p.L, dt=p.dt, tol=1e-14, max_cycles=1500, adj_tol=1e-13)
    phi0 = dev(inputs.adjoint_phi0(64, seed=5))
    with torch.no_grad():
        tgt = rollout(dev(inputs.adjoint_phi0(64, seed=6)), torch.tensor(0.12, dtype=torch.float64),
                      params, p.steps)

    def final(ph, eps):
        with torch.no_grad():
            return rollout(ph, torch.tensor(eps, dtype=torch.float64), params, p.steps)

    def loss_diff(a, b):
        # L(a) - L(b) for L = sum (phi_T - target)^2, written as
        # sum (a - b)(a + b - 2 target): no cancellation between two large sums
        return float(((a - b) * (a + b - 2.0 * tgt)).sum())

    p0 = phi0.clone().requires_grad_(True)
    e = torch.tensor(p.eps, dtype=torch.float64, requires_grad=True)
    out = rollout(p0, e, params, p.steps, ckpt_every=5)
    loss = ((out - tgt) ** 2).sum()
    loss.backward()
    v = dev(inputs.unit_direction((64, 64, 64), seed=7))
    d = 1e-6
    fd = loss_diff(final(phi0 + d * v, p.eps), final(phi0 - d * v, p.eps)) / (2 * d)
    ad = float((p0.grad * v).sum())
    print(f"directional derivative: adjoint {ad:.12e} FD {fd:.12e} rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= 1e-6 * abs(fd)
    fde = loss_diff(final(phi0, p.eps + d), final(phi0, p.eps - d)) / (2 * d)
    print(f"d/deps: adjoint {float(e.grad):.12e} FD {fde:.12e} rel {abs(float(e.grad) - fde) / abs(fde):.2e}")
    assert abs(float(e.grad) - fde) <= 1e-6 * abs(fde)


@pytest.mark.parametrize("n", [32, 64])
def test_recompute_reproduces_the_forward_segment_bitwise(n):
    """Checkpoint-and-recompute: the backward pass recomputes each segment
    from its checkpoint after other work has run on the handle (later
    segments, adjoint steps, unrelated steps that leave another coarsest
    inverse in the cache).  run_segment clears the cache first, so the
    recomputed trajectory must equal the forward one bit for bit."""
    from paper_1611_06288_amd import Solver
    from paper_1611_06288_amd.autograd import run_segment
    p = inputs.adjoint_params(n)
    s = Solver(n, p.L, p.eps, p.dt, tol=1e-12, max_cycles=600)
    phi0 = dev(inputs.adjoint_phi0(n, seed=5))
    mu, om = s.init_guess(phi0)
    state = (phi0.clone(), phi0.clone(), mu, om)
    fwd, ckpts = [], []
    for seg in range(2):
        ckpts.append(tuple(t.clone() for t in state))
        phis, mu, om = run_segment(s, state, 5)
        fwd.append(([t.clone() for t in phis], mu.clone(), om.clone()))
        state = (phis[-2], phis[-1], mu, om)
    # disturb the cache: steps on another field, and an adjoint step
    other = dev(inputs.adjoint_phi0(n, seed=9))
    mu2, om2 = s.init_guess(other)
    s.step(other, other, mu2, om2)
    g = torch.zeros_like(phi0)
    geps = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.adjoint_step(fwd[1][0][0], fwd[1][0][1], fwd[1][0][2], other, g, g, geps)
    for seg in (1, 0):
        phis, mu_r, om_r = run_segment(s, ckpts[seg], 5)
        want, mu_w, om_w = fwd[seg]
        for k, (a, b) in enumerate(zip(phis, want)):
            assert torch.equal(a, b), (seg, k, float((a - b).abs().max()))
        assert torch.equal(mu_r, mu_w) and torch.equal(om_r, om_w), seg

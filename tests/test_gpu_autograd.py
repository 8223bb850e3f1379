"""Differentiation form: autograd through the adjoint kernels.

* a directional check of dL/dD, dL/dtau, dL/deps on a tiny cell against
  central differences of the forward GPU density, and torch.autograd.gradcheck
  of rho(D, tau, eps) there (D in a random subspace);
* on the 868-atom bilayer (the benchmark geometry): dE/dtau on 10 random
  atoms and the full strain derivative against central finite differences
  (dR = 1e-4 Bohr, strain 1e-5) of the FP64 GPU energy, and against the
  oracle's analytic force.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def test_rho_vjp_tiny(torch_dev):
    from paper_2409_09399_amd import autograd as A
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(4, grid=(12, 12, 12))
    rng = np.random.default_rng(0)
    d = torch.tensor(s.d, device=dev, requires_grad=True)
    tau = torch.tensor(s.pos, device=dev, requires_grad=True)
    eps = torch.zeros(3, 3, dtype=torch.float64, device=dev, requires_grad=True)
    g = torch.tensor(rng.normal(size=s.ngrid), device=dev)
    L = torch.dot(A.rho(s, d, tau, eps), g)
    L.backward()

    def Lval(dd=None, tt=None, ee=None):
        with torch.no_grad():
            r = A.rho(s, d if dd is None else dd, tau if tt is None else tt, eps if ee is None else ee)
            return float(torch.dot(r, g))

    # D: linear, one directional derivative is exact
    u = torch.tensor(rng.normal(size=s.nnz), device=dev)
    fd = Lval(dd=d.detach() + u) - Lval(dd=d.detach())
    assert abs(fd - float(torch.dot(d.grad, u))) <= 1e-9 * max(1.0, abs(fd))
    h = 1e-4
    for K, a in ((0, 0), (3, 2), (6, 1)):
        tp = tau.detach().clone(); tp[K, a] += h
        tm = tau.detach().clone(); tm[K, a] -= h
        fd = (Lval(tt=tp) - Lval(tt=tm)) / (2 * h)
        assert abs(fd - float(tau.grad[K, a])) <= 2e-6 * float(tau.grad.abs().max()), (K, a)
    he = 1e-5
    for a, b in ((0, 0), (1, 2), (2, 0)):
        ep = torch.zeros(3, 3, dtype=torch.float64, device=dev); ep[a, b] = he
        fd = (Lval(ee=ep) - Lval(ee=-ep)) / (2 * he)
        assert abs(fd - float(eps.grad[a, b])) <= 2e-6 * float(eps.grad.abs().max()), (a, b)


def test_rho_gradcheck_tiny(torch_dev):
    """torch.autograd.gradcheck of rho(D, tau, eps) in FP64 on the tiny cell:
    D moves in a random three-dimensional subspace (the full nnz would take a
    forward pass per entry), tau and eps in full, rho projected onto four
    random vectors; the Jacobian from the adjoint kernels must match central
    differences entry by entry."""
    from paper_2409_09399_amd import autograd as A
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(4, grid=(12, 12, 12))
    rng = np.random.default_rng(3)
    d0 = torch.tensor(s.d, device=dev)
    U = torch.tensor(rng.normal(size=(3, s.nnz)) * np.abs(s.d).max(), device=dev)
    Pm = torch.tensor(rng.normal(size=(s.ngrid, 4)), device=dev)

    def f(c, tau, eps):
        return A.rho(s, d0 + c @ U, tau, eps) @ Pm

    c = torch.zeros(3, dtype=torch.float64, device=dev, requires_grad=True)
    tau = torch.tensor(s.pos, device=dev, requires_grad=True)
    eps = torch.zeros(3, 3, dtype=torch.float64, device=dev, requires_grad=True)
    # nondet_tol: the FP64 atomics of the adjoint kernels may add in another
    # order on a second backward pass
    assert torch.autograd.gradcheck(f, (c, tau, eps), eps=1e-6, atol=1e-7, rtol=1e-5, nondet_tol=1e-10)


def test_energy_fd_tbg868(torch_dev, oracle_mod):
    from paper_2409_09399_amd import autograd as A
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.make_config(2)
    v = torch.tensor(s.v, device=dev)
    d = torch.tensor(s.d, device=dev)
    tau = torch.tensor(s.pos, device=dev, requires_grad=True)
    eps = torch.zeros(3, 3, dtype=torch.float64, device=dev, requires_grad=True)
    E = A.energy(s, v, d, tau, eps)
    E.backward()
    gtau = tau.grad.cpu().numpy()
    geps = eps.grad.cpu().numpy()
    rng = np.random.default_rng(0)
    atoms = rng.choice(s.natom, 10, replace=False)

    def Eval(tt=None, ee=None):
        with torch.no_grad():
            return float(A.energy(s, v, d, tau.detach() if tt is None else tt,
                                  eps.detach() if ee is None else ee))

    h = 1e-4
    fscale = np.abs(gtau).max()
    worst = 0.0
    for K in atoms:
        for a in range(3):
            tp = tau.detach().clone(); tp[K, a] += h
            tm = tau.detach().clone(); tm[K, a] -= h
            fd = (Eval(tt=tp) - Eval(tt=tm)) / (2 * h)
            worst = max(worst, abs(fd - gtau[K, a]) / fscale)
    print("[autograd] force FD worst rel", worst, flush=True)
    assert worst <= 1e-6
    he = 1e-5
    sworst = 0.0
    for a in range(3):
        for b in range(3):
            ep = torch.zeros(3, 3, dtype=torch.float64, device=dev); ep[a, b] = he
            fd = (Eval(ee=ep) - Eval(ee=-ep)) / (2 * he)
            sworst = max(sworst, abs(fd - geps[a, b]) / np.abs(geps).max())
    print("[autograd] strain FD worst rel", sworst, flush=True)
    assert sworst <= 1e-6
    # and against the oracle's analytic force: dE/dtau = -F
    Fo, _ = oracle_mod.Oracle(s).force_atoms(atoms[:4])
    assert np.abs(-gtau[atoms[:4]] - Fo).max() <= 1e-10 * np.abs(Fo).max()


def test_energy_from_library_and_plan_reuse(torch_dev):
    """The energy is the library's reduction (equal to the force pass's E
    and to sum w V rho), the plan is reused at fixed geometry, and backward
    can run twice with retain_graph."""
    from paper_2409_09399_amd import autograd as A
    from paper_2409_09399_amd import gint as G
    from paper_2409_09399_amd import inputs as I
    torch, dev = torch_dev
    s = I.diamond8(2, grid=(16, 16, 16))
    v = torch.tensor(s.v, device=dev)
    d = torch.tensor(s.d, device=dev, requires_grad=True)
    tau = torch.tensor(s.pos, device=dev, requires_grad=True)
    E = A.energy(s, v, d, tau)
    plan1 = A._plan_cache["entry"][2]
    E2 = A.energy(s, v, d, tau)
    assert A._plan_cache["entry"][2] is plan1          # same geometry: plan reused
    # rho is accumulated with FP64 atomics, so two calls agree to rounding
    # (the order of the additions varies), not bit for bit
    assert abs(float(E) - float(E2)) <= 1e-13 * abs(float(E2))
    plan = G.Plan(s)
    F = torch.empty(3 * s.natom, dtype=torch.float64, device=dev)
    sig = torch.empty(9, dtype=torch.float64, device=dev)
    Ef = torch.empty(1, dtype=torch.float64, device=dev)
    G.gint_force_stress(plan, v, d.detach(), F, sig, Ef)
    torch.cuda.synchronize()
    assert abs(float(E) - float(Ef[0])) <= 1e-12 * abs(float(Ef[0]))
    E.backward(retain_graph=True)
    g1 = tau.grad.clone()
    tau.grad = None
    E.backward()
    # the force kernel reduces with atomics too: equal to rounding
    assert torch.allclose(g1, tau.grad, rtol=0, atol=1e-13 * float(g1.abs().max()))
    assert torch.allclose(-g1.reshape(-1), F, rtol=0, atol=1e-12 * float(F.abs().max()))
    plan.close()

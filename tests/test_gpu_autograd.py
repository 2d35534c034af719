"""Differentiation through the GPU transforms, operator and solve.

* SHTSynth / SHTAdjoint / ApplyA backward equals the transposed operator
  computed by the oracle (the backward of a linear map is its transpose).
* CRSolve: dL/db and dL/dq_beta (C_l = q_beta C_fid_l on log bands) for
  L = 1/2 ||x||^2 against central finite differences (rebuilding operator and
  solver for q +- eps; b held fixed), on the dense direct solve (N_side 16)
  and on the multi-level W-cycle (N_side 256), and against the closed form
  with N^-1 = 0 (x = S b: dL/db = S^2 b, dL/dq_beta = sum_beta C_l^2 b^2 at q = 1).
"""
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import operator as oop
from oracle import sht as osht
from tests.gpu_util import dev, host, parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


def test_linear_maps_backward(mlcr):
    from paper_1308_5299_amd.autograd import ApplyA, SHTAdjoint, SHTSynth
    cfg = workloads.get_config("c1")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    rng = np.random.default_rng(41)
    x = dev(rng.standard_normal((2, cfg.nalm))).requires_grad_(True)
    w = rng.standard_normal((2, cfg.npix))
    (SHTSynth.apply(x, g, cfg.lmax, mlcr.FP64) * dev(w)).sum().backward()
    assert parity(host(x.grad), osht.adjoint(w, cfg.lmax, cfg.nside)) <= 1e-12
    y = dev(w).requires_grad_(True)
    v = rng.standard_normal((2, cfg.nalm))
    (SHTAdjoint.apply(y, g, cfg.lmax, mlcr.FP64) * dev(v)).sum().backward()
    assert parity(host(y.grad), osht.synth(v, cfg.lmax, cfg.nside)) <= 1e-12
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=2)
    x2 = dev(rng.standard_normal((2, cfg.nalm))).requires_grad_(True)
    (ApplyA.apply(x2, op, 0, mlcr.FP64) * dev(v)).sum().backward()
    assert parity(host(x2.grad), oop.apply_A(v, d["cl"], d["bl"], d["ninv"], cfg.nside)) <= 1e-12


def _loss_and_grads(mlcr, cfg, d, cl_fid, q, edges, b, ninv, rtol):
    from paper_1308_5299_amd.autograd import band_index, cr_solve
    band = band_index(cfg.lmax, edges)
    cl = cl_fid.copy()
    cl[band >= 0] *= q[band[band >= 0]]
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, cl, d["bl"], ninv, max_nrhs=1)
    S = mlcr.Solver(op, max_nrhs=1)
    bt = dev(b).requires_grad_(True)
    qt = torch.tensor(q, dtype=torch.float64, device="cuda", requires_grad=True)
    x = cr_solve(bt, S, qt, cl_fid, edges, rtol=rtol, max_cycles=80)
    L = 0.5 * (x * x).sum()
    L.backward()
    return float(L.detach()), host(bt.grad), host(qt.grad)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_crsolve_gradients_finite_differences(mlcr, name):
    from paper_1308_5299_amd.autograd import log_bands
    print(f"case crsolve gradients {name}", flush=True)
    cfg = workloads.get_config(name)
    d = workloads.workload_inputs(cfg)
    cl_fid = d["cl"].copy()
    edges = log_bands(cfg.lmax, 64)
    nb = len(edges) - 1
    q = np.ones(nb)
    ninv = dev(d["ninv"])
    rng = np.random.default_rng(51)
    b = osht.adjoint(d["ninv"][None] * rng.standard_normal((1, cfg.npix)), cfg.lmax, cfg.nside)
    rtol = 1e-12
    L0, gb, gq = _loss_and_grads(mlcr, cfg, d, cl_fid, q, edges, b, ninv, rtol)
    # dL/db along a random direction
    dvec = rng.standard_normal(b.shape)
    eps = 1e-3 * np.linalg.norm(b) / np.linalg.norm(dvec)
    Lp = _loss_and_grads(mlcr, cfg, d, cl_fid, q, edges, b + eps * dvec, ninv, rtol)[0]
    Lm = _loss_and_grads(mlcr, cfg, d, cl_fid, q, edges, b - eps * dvec, ninv, rtol)[0]
    fd = (Lp - Lm) / (2 * eps)
    an = float(np.sum(gb * dvec))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # dL/dq for a low, a middle and the top band
    for beta in [0, nb // 2, nb - 1]:
        h = 1e-4
        qp, qm = q.copy(), q.copy()
        qp[beta] += h
        qm[beta] -= h
        Lp = _loss_and_grads(mlcr, cfg, d, cl_fid, qp, edges, b, ninv, rtol)[0]
        Lm = _loss_and_grads(mlcr, cfg, d, cl_fid, qm, edges, b, ninv, rtol)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gq[beta]) <= 1e-6 * max(abs(fd), 1e-12 * abs(L0)), (beta, fd, gq[beta])


def test_crsolve_gradient_closed_form(mlcr):
    """N^-1 = 0: A = S^-1, x = S b; dL/db = S^2 b, dL/dq_beta = sum C_l^2 b^2.
    The prior is made positive at l < 2 too, else A would be singular there."""
    from paper_1308_5299_amd.autograd import band_index, log_bands
    cfg = workloads.get_config("c1")
    d = workloads.workload_inputs(cfg)
    cl = d["cl"].copy()
    cl[:2] = cl[2]
    edges = log_bands(cfg.lmax, 64)
    ninv0 = dev(np.zeros(cfg.npix))
    b = np.random.default_rng(61).standard_normal((1, cfg.nalm))
    L0, gb, gq = _loss_and_grads(mlcr, cfg, d, cl, np.ones(len(edges) - 1), edges, b, ninv0, 1e-14)
    C = cl[workloads.packed_ell(cfg.lmax)]
    np.testing.assert_allclose(gb[0], C * C * b[0], rtol=1e-12, atol=0)
    band = band_index(cfg.lmax, edges)[workloads.packed_ell(cfg.lmax)]
    want = np.array([np.sum((C * C * b[0] * b[0])[band == k]) for k in range(len(edges) - 1)])
    np.testing.assert_allclose(gq, want, rtol=1e-12, atol=0)


@pytest.mark.timeout(900)
def test_c5_gradients_finite_differences(mlcr):
    """Differentiation at full scale (N_side 2048 / lmax 4096): dL/db along a
    random direction and dL/dq_beta for a low, a middle and the top of the 64
    log bands, for L = 1/2 ||x||^2, against central finite differences.  The
    perturbed systems are solved with the hierarchy built at q = 1 after
    mlcr_op_set_prior (the float64 residual carries the new C_l); every solve
    runs bf16x3 cycles with float64 refinement to rho <= 1e-13 or better."""
    from paper_1308_5299_amd.autograd import band_index, cr_solve, log_bands
    print("case c5 gradients vs finite differences", flush=True)
    cfg = workloads.get_config("c5")
    d = workloads.workload_inputs(cfg)
    cl_fid = d["cl"].copy()
    edges = log_bands(cfg.lmax, 64)
    nb = len(edges) - 1
    band = band_index(cfg.lmax, edges)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    ninv = dev(d["ninv"])
    op = mlcr.Operator(g, cl_fid, d["bl"], ninv, max_nrhs=1)
    t0 = time.time()
    S = mlcr.Solver(op, max_nrhs=1)
    torch.cuda.synchronize()
    print(f"setup {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(52)
    b = mlcr.sht_adjoint(g, ninv * dev(rng.standard_normal((1, cfg.npix))))
    prec, rtol = mlcr.BF16X3, 1e-13

    def loss(bv):
        x, info = S.solve(bv, rtol=rtol, max_cycles=40, prec=prec, raise_on_noconv=False)
        assert info[0]["rho"] <= 1e-12, info[0]
        return 0.5 * float((x * x).sum())

    bt = b.clone().requires_grad_(True)
    qt = torch.ones(nb, dtype=torch.float64, device="cuda", requires_grad=True)
    t0 = time.time()
    x = cr_solve(bt, S, qt, cl_fid, edges, rtol=rtol, max_cycles=40, prec=prec)
    L0 = 0.5 * (x * x).sum()
    L0.backward()
    L0 = float(L0.detach())
    gb, gq = bt.grad.detach(), host(qt.grad)
    print(f"forward + backward {time.time() - t0:.1f}s, L = {L0:.6e}", flush=True)
    dvec = dev(rng.standard_normal((1, cfg.nalm)))
    eps = 1e-3 * float(b.norm() / dvec.norm())
    fd = (loss(b + eps * dvec) - loss(b - eps * dvec)) / (2 * eps)
    an = float((gb * dvec).sum())
    print(f"dL/db . d: analytic {an:.10e}, central FD {fd:.10e}", flush=True)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    h = 1e-4
    for beta in [0, nb // 2, nb - 1]:
        Ls = []
        for sgn in (1.0, -1.0):
            cl = cl_fid.copy()
            cl[band == beta] *= 1.0 + sgn * h
            op.set_prior(cl)
            Ls.append(loss(b))
        op.set_prior(cl_fid)
        fdq = (Ls[0] - Ls[1]) / (2 * h)
        print(f"band {beta} (l {edges[beta]}..{edges[beta + 1] - 1}): analytic {gq[beta]:.10e}, "
              f"central FD {fdq:.10e}", flush=True)
        assert abs(fdq - gq[beta]) <= 1e-6 * max(abs(fdq), 1e-12 * abs(L0)), (beta, fdq, gq[beta])

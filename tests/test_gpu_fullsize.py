"""Full-size checks in the launch configuration the benchmark times
(N_side 2048, lmax 4096, 8 RHS per launch), and the multi-level solves at
N_side 1024 / lmax 2048 and N_side 2048 / lmax 4096 in all three precisions.

At N_side 2048 the oracle cannot run whole transforms, so it is asked for
samples it computes one by one:
* synthesis: every pixel of whole rings, one or more from every ring-FFT
  launch group (power-of-two and Bluestein lengths, the 512- and 1024-thread
  launches, north and south caps, belt);
* adjoint: whole orders m from many 8-order work groups (direct trigonometric
  ring sums, all rings).
The operator is then checked through properties that hold at any size:
symmetry <u, A v> = <A u, v>; the fused ring kernel equals the composition
of the sampled-checked transforms; the mixed paths stay within their
rounding bounds of the float64 path.

Solves use manufactured solutions b = A x_true (Sec. 4.1).  At N_side 1024
the oracle computes b, the max pixel error over all pixels and the
certificate of every solution.  At N_side 2048 b comes from the float64
apply (checked above on samples) and the error is measured by the oracle on
sampled rings and by the float64 synthesis over all pixels.  Every parity
bar applies both to the relative 2-norm and to max |y - y_ref| / max |y_ref|
(for the float64 path at lmax 4096 the per-element bar is scaled by
lmax / 512, see tests/gpu_util.elem_bar).
"""
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import operator as oop
from oracle import sht as osht
from oracle import solve as osolve
from tests.gpu_util import check, dev, host, parity

pytestmark = pytest.mark.gpu

R = 8
TOL = 1e-12
TOL32 = 2e-5          # float32 contraction: ~2^-24 sqrt(lmax) relative
TOLB3 = 1e-4          # split-bfloat16 contraction: 3 * 2^-18 per product, 9x margin


def _check(got, want, tol, fp64, slack=1.0):
    return check(got, want, tol, 4096, fp64, slack)


# Rings (0-based RING index k, ring i = k + 1) covering every launch group of
# the ring kernel at N_side 2048.  The complex FFT of a ring of N = 4i pixels
# has n = 2i points; n a power of two runs radix-8 passes, else Bluestein of
# size M = the power of two >= 2n - 1.  Groups: M <= 1024, 2048, 4096 (512
# threads) and 8192 (1024 threads); rings of <= 1024 pixels fold cooperatively.
C5_RINGS = [
    0,      # i = 1, N = 4 (pole), power of two
    2,      # i = 3, Bluestein M = 16
    255,    # i = 256, power of two n = 512
    299,    # i = 300, Bluestein M = 2048 (512 threads)
    511,    # i = 512, power of two n = 1024
    700,    # i = 701, Bluestein M = 4096 (512 threads)
    1023,   # i = 1024, power of two n = 2048
    1500,   # i = 1501, Bluestein M = 8192 (1024 threads)
    2046,   # i = 2047, last cap ring, Bluestein M = 8192
    2047,   # first belt ring, n = 4096
    3000,   # belt
    4095,   # equator
    6143,   # last belt ring
    6144,   # first south-cap ring (mirror of i = 2047)
    7890,   # south cap, mirror of i = 301, Bluestein M = 2048
    8190,   # south pole ring
]
# Orders from many 8-order work groups (the Legendre kernels run groups of 8
# consecutive orders side by side), including both ends of groups and the
# shortest orders.
C5_ORDERS = [0, 1, 7, 8, 9, 15, 16, 100, 511, 777, 1500, 2048, 2049, 3001, 4000, 4090, 4095, 4096]


@pytest.fixture(scope="module")
def mlcr():
    import paper_1308_5299_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def c5(mlcr):
    cfg = workloads.get_config("c5")
    d = workloads.workload_inputs(cfg)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    x = np.stack([workloads.prior_sample(cfg, r) for r in range(R)])
    return cfg, d, g, x


def _ring_values(maps, geo, rings):
    return {k: host(maps[:, geo.start[k]: geo.start[k] + geo.nphi[k]]) for k in rings}


def test_c5_synthesis_sampled_rings(mlcr, c5):
    cfg, d, g, x = c5
    print(f"case c5 synthesis, 8 RHS, {len(C5_RINGS)} sampled rings", flush=True)
    geo = osht.healpix_rings(cfg.nside)
    t0 = time.time()
    ref = osht.synth_rings(x, cfg.lmax, cfg.nside, C5_RINGS)
    print(f"oracle rings in {time.time() - t0:.1f}s", flush=True)
    allr = np.concatenate([ref[k] for k in C5_RINGS], axis=1)
    # the bar applies to the sampled output as a whole; a single polar ring
    # holds only a few pixels, so single rings get 4x slack
    for prec, tol in [(mlcr.FP64, TOL), (mlcr.FP32, TOL32), (mlcr.BF16X3, TOLB3)]:
        f = mlcr.sht_synth(g, dev(x), prec=prec)
        got = _ring_values(f, geo, C5_RINGS)
        del f
        allg = np.concatenate([got[k] for k in C5_RINGS], axis=1)
        per = {k: parity(got[k], ref[k]) for k in C5_RINGS}
        ok, (e2, em) = _check(allg, allr, tol, prec == mlcr.FP64)
        print(f"prec {prec}: sampled rings rel2 {e2:.2e} max-elem {em:.2e}, worst ring "
              f"{max(per, key=per.get)} {max(per.values()):.2e}", flush=True)
        assert ok, (prec, e2, em)
        for k in C5_RINGS:
            assert _check(got[k], ref[k], tol, prec == mlcr.FP64, slack=4.0)[0], (prec, k, per[k])


def test_c5_adjoint_sampled_orders(mlcr, c5):
    cfg, d, g, x = c5
    print(f"case c5 adjoint, 8 RHS, {len(C5_ORDERS)} sampled orders", flush=True)
    y = np.random.default_rng(77).standard_normal((R, cfg.npix))
    t0 = time.time()
    ref = osht.adjoint_orders(y, cfg.lmax, cfg.nside, C5_ORDERS)
    print(f"oracle orders in {time.time() - t0:.1f}s", flush=True)
    for prec, tol in [(mlcr.FP64, TOL), (mlcr.FP32, TOL32), (mlcr.BF16X3, TOLB3)]:
        a = mlcr.sht_adjoint(g, dev(y), prec=prec)
        got, want = [], []
        for m in C5_ORDERS:
            c, s = ref[m]
            if m == 0:
                got.append(host(a[:, : cfg.lmax + 1]))
                want.append(c)
                continue
            b = osht.block_base(m, cfg.lmax)
            n = cfg.lmax - m + 1
            got += [host(a[:, b: b + n]), host(a[:, b + n: b + 2 * n])]
            want += [c, s]
        del a
        per = [parity(u, v) for u, v in zip(got, want)]
        ok, (e2, em) = _check(np.concatenate(got, axis=1), np.concatenate(want, axis=1), tol,
                              prec == mlcr.FP64)
        print(f"prec {prec}: sampled orders rel2 {e2:.2e} max-elem {em:.2e}, worst block "
              f"{max(per):.2e}", flush=True)
        # bar over the sampled output as a whole; the m = lmax blocks hold a
        # single coefficient each, so blocks get 4x slack
        assert ok, (prec, e2, em)
        for u, v in zip(got, want):
            assert _check(u, v, tol, prec == mlcr.FP64, slack=4.0)[0], (prec, per)


def test_c5_apply_properties(mlcr, c5):
    cfg, d, g, x = c5
    print("case c5 apply_A properties, 8 RHS", flush=True)
    ninv = dev(d["ninv"])
    op = mlcr.Operator(g, d["cl"], d["bl"], ninv, max_nrhs=R)
    u = dev(x)
    v = dev(np.stack([workloads.prior_sample(cfg, R + r) for r in range(R)]))
    Au = mlcr.apply_A(op, u)
    Av = mlcr.apply_A(op, v)
    # symmetry, per RHS
    lhs = (u * Av).sum(dim=1)
    rhs = (Au * v).sum(dim=1)
    assert float(((lhs - rhs).abs() / lhs.abs()).max()) <= 1e-12
    # the fused ring step equals synthesis -> N^-1 -> adjoint, plus the prior
    L = workloads.packed_ell(cfg.lmax)
    bl = dev(d["bl"][L])
    sinv = dev(np.where(d["cl"][L] > 0, 1.0 / np.where(d["cl"][L] > 0, d["cl"][L], 1.0), 0.0))
    mp = mlcr.sht_synth(g, bl * u)
    comp = sinv * u + bl * mlcr.sht_adjoint(g, mp * ninv)
    del mp
    assert _check(host(comp), host(Au), TOL, True)[0]
    # mixed paths within their rounding bounds of the float64 path
    Au_h = host(Au)
    e32 = parity(host(mlcr.apply_A(op, u, prec=mlcr.FP32)), Au_h)
    eb3 = parity(host(mlcr.apply_A(op, u, prec=mlcr.BF16X3)), Au_h)
    print(f"apply vs float64: fp32 {e32:.2e}, bf16x3 {eb3:.2e}", flush=True)
    assert e32 <= TOL32
    assert eb3 <= TOLB3


def _precs(mlcr):
    return {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}


@pytest.mark.timeout(900)
def test_c3_solves_anchored_on_oracle(mlcr):
    """8 RHS at N_side 1024 / lmax 2048 in fp64, fp32 and bf16x3: b = A x_true
    by the oracle's float64 apply; every solution judged by the oracle's max
    pixel error over all pixels (<= 1e-3 uK) and by the oracle's certificate
    sigma_prior ||S^{1/2}(b - A x)||, which must bound that error."""
    cfg = workloads.get_config("c3")
    d = workloads.workload_inputs(cfg)
    cl, bl = d["cl"], d["bl"]
    print("case c3 solves, 8 RHS, oracle-manufactured b", flush=True)
    xt = np.stack([workloads.prior_sample(cfg, r) for r in range(R)])
    t0 = time.time()
    b = osolve.manufactured(xt, cl, bl, d["ninv"], cfg.nside)
    print(f"oracle b in {time.time() - t0:.1f}s", flush=True)
    g = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(g, cl, bl, dev(d["ninv"]), max_nrhs=R)
    S = mlcr.Solver(op, max_nrhs=R)
    bd = dev(b)
    xs, cycles = [], {}
    for name, prec in _precs(mlcr).items():
        torch.cuda.synchronize()
        t0 = time.time()
        x, info = S.solve(bd, rtol=1e-7, max_cycles=30, prec=prec)
        torch.cuda.synchronize()
        cycles[name] = [i["cycles"] for i in info]
        print(f"c3 {name}: cycles {cycles[name]}, {time.time() - t0:.2f} s", flush=True)
        assert all(i["converged"] == 1 for i in info), name
        xs.append(host(x))
    X = np.concatenate(xs)                          # [3 R, nalm]
    XT = np.concatenate([xt] * 3)
    t0 = time.time()
    err = np.abs(osht.synth(X - XT, cfg.lmax, cfg.nside)).max(axis=1)
    print(f"oracle errors in {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    act = osolve.active_modes(cl)
    res = np.where(act, np.concatenate([b] * 3) - oop.apply_A(X, cl, bl, d["ninv"], cfg.nside), 0.0)
    Ld = oop.mode_ell(cfg.lmax)
    bound = osolve.sigma_prior(cl) * np.linalg.norm(np.sqrt(cl[Ld]) * res, axis=1)
    print(f"oracle certificates in {time.time() - t0:.1f}s", flush=True)
    for j, name in enumerate(_precs(mlcr)):
        e, bd_ = err[j * R:(j + 1) * R], bound[j * R:(j + 1) * R]
        print(f"c3 {name}: max pixel error {e.max():.3e} uK, certificate {bd_.max():.3e} uK", flush=True)
        assert e.max() <= 1e-3, (name, e)
        assert np.all(e <= bd_ * (1 + 1e-9)), (name, e, bd_)


@pytest.mark.timeout(900)
def test_c5_solves_to_1e3_uK(mlcr, c5):
    """8 RHS at N_side 2048 / lmax 4096 in fp64, fp32 and bf16x3: W-cycles on
    b = A x_true (float64 apply) reach 1e-3 uK max pixel error, measured by the
    float64 synthesis over all pixels and by the oracle on sampled rings of
    every ring-FFT launch group."""
    cfg, d, g, xt = c5
    print("case c5 solves, 8 RHS", flush=True)
    op = mlcr.Operator(g, d["cl"], d["bl"], dev(d["ninv"]), max_nrhs=R)
    t0 = time.time()
    S = mlcr.Solver(op, max_nrhs=R)
    torch.cuda.synchronize()
    print(f"setup {time.time() - t0:.1f}s", flush=True)
    xtd = dev(xt)
    b = mlcr.apply_A(op, xtd)
    errs = []
    for name, prec in _precs(mlcr).items():
        torch.cuda.synchronize()
        t0 = time.time()
        x, info = S.solve(b, rtol=0.0, max_cycles=9, prec=prec, raise_on_noconv=False)
        torch.cuda.synchronize()
        dt = time.time() - t0
        e_all = float(mlcr.sht_synth(g, x - xtd).abs().max())
        print(f"c5 {name}: 9 cycles {dt:.2f} s, rho {max(i['rho'] for i in info):.2e}, "
              f"max pixel error (float64 synthesis, all pixels) {e_all:.3e} uK", flush=True)
        assert e_all <= 1e-3, (name, e_all)
        errs.append(host(x) - xt)
        del x
    rings = [0, 299, 700, 1500, 4095, 7890]
    t0 = time.time()
    ref = osht.synth_rings(np.concatenate(errs), cfg.lmax, cfg.nside, rings)
    print(f"oracle rings in {time.time() - t0:.1f}s", flush=True)
    for j, name in enumerate(_precs(mlcr)):
        e = max(float(np.abs(ref[k][j * R:(j + 1) * R]).max()) for k in rings)
        print(f"c5 {name}: max error on oracle-sampled rings {e:.3e} uK", flush=True)
        assert e <= 1e-3, (name, e)


@pytest.mark.parametrize("nrhs", [1, 2])
def test_adjoint_ignores_stale_workspace(mlcr, nrhs):
    """Regression: the vector adjoint's split-K chunks each store their
    partial sums; no chunk may be left empty (its slice would be stale when a
    larger transform used the workspace before).  N_side 300 / lmax 2048 has 5
    ring-pair blocks, the shape that once produced an empty chunk."""
    print(f"case stale workspace nrhs={nrhs}", flush=True)
    nside, lmax = 300, 2048
    g = mlcr.Geometry(nside, lmax)
    y = dev(np.random.default_rng(88).standard_normal((nrhs, 12 * nside * nside)))
    a1 = mlcr.sht_adjoint(g, y).clone()
    big = dev(np.random.default_rng(89).standard_normal((16, 12 * nside * nside)))
    mlcr.sht_adjoint(g, big)                 # fills the workspaces with other data
    del big
    a2 = mlcr.sht_adjoint(g, y)
    assert torch.equal(a1, a2)
    # and against the oracle on a few whole orders
    ref = osht.adjoint_orders(host(y), lmax, nside, [0, 700, 2048])
    got = [host(a2[:, : lmax + 1])]
    want = [ref[0][0]]
    for m in (700, 2048):
        b = osht.block_base(m, lmax)
        n = lmax - m + 1
        got += [host(a2[:, b: b + n]), host(a2[:, b + n: b + 2 * n])]
        want += [ref[m][0], ref[m][1]]
    assert parity(np.concatenate(got, axis=1), np.concatenate(want, axis=1)) <= TOL

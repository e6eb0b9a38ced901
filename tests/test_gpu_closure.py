"""GPU parity of the learned closure's kernels against the FP64 oracle (with bfloat16 emulation),
and a small training run that must beat the plain 1x force on held-out data.

Tolerances: the forward output and the weight
gradients (two tiles per workgroup of the weight-gradient kernel at 32^3) are compared in relative L2; bfloat16 has a unit roundoff of 2^-9,
and an occasional one-ulp difference in a rounded activation (FP32 versus FP64
accumulation right at a rounding boundary) perturbs the output by about that
much at a handful of points, so 2e-3 bounds the output and 2e-2 the gradients
(which pass through three bfloat16 roundings of back-propagated values).
"""
import numpy as np
import pytest

from oracle import cnn
from oracle import pm as opm
from synth import config_particles, spectrum_power_law_m2
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup():
    from paper_2607_17929_amd import PMContext
    pos, u, tau0, _ = config_particles("zeldovich_32_scalar_fp64")
    n = 32
    ctx = PMContext(n, pos.shape[0], 320.0, physics="scalar", precision="fp64", closure=True)
    ctx.init_particles(pos, u, tau0)
    ctx.deposit()
    ctx.solve_metric(0.0)
    sim = opm.OracleSim(n=n, box_mpch=320.0, physics="scalar", pos=pos, u=u, tau=tau0)
    sim.deposit()
    n00 = sim.dep[0].copy()
    sim.solve(0.0)
    return ctx, sim, n00, opm.wrap_positions(pos.copy()), n


def _params(seed=3):
    r = np.random.default_rng(seed)
    p = 0.15 * r.standard_normal(cnn.N_PARAMS)
    return p.astype(np.float32).astype(np.float64)


def test_closure_forward_and_backward_parity():
    print("closure parity", flush=True)
    ctx, sim, n00, pos, n = _setup()
    params = _params()
    ctx.closure_set_params(torch.tensor(params, dtype=torch.float32))
    ctx.closure_forward(False)
    out = ctx.closure_gather().cpu().numpy().astype(np.float64)
    x, rms = cnn.features(n00, sim.phi)
    y, acts = cnn.forward(params, x)
    ref = cnn.gather(y, pos)
    assert abs(ctx.closure_scale() - rms) < 1e-6 * rms
    e = rel_l2(out, ref)
    print("forward rel-L2", e, flush=True)
    assert e < 2e-3
    r = np.random.default_rng(5)
    dpred = r.standard_normal((pos.shape[0], 3)).astype(np.float32)
    g = ctx.closure_backward(torch.tensor(dpred)).cpu().numpy().astype(np.float64)
    d3 = cnn.gather_adjoint(dpred.astype(np.float64), pos, n)
    gref = cnn.backward(params, acts, d3)
    offs = [0, 16 * 4 * 27 + 16, 16 * 4 * 27 + 16 + 16 * 16 * 27 + 16, cnn.N_PARAMS]
    for k in range(3):
        ek = rel_l2(g[offs[k]:offs[k + 1]], gref[offs[k]:offs[k + 1]])
        print(f"layer {k + 1} gradient rel-L2 {ek:.3e}", flush=True)
        assert ek < 2e-2


def test_closure_loss_against_oracle():
    """pm_closure_loss: the residual of the gathered output against a target, its MSE gradient and the two
    FP64 means, against the oracle's MSE on the same prediction (the GPU forms the residual in FP32)."""
    print("closure loss", flush=True)
    ctx, sim, n00, pos, n = _setup()
    ctx.closure_set_params(torch.tensor(_params(), dtype=torch.float32))
    ctx.closure_forward(False)
    pred = ctx.closure_gather().cpu().numpy()
    target = np.random.default_rng(11).standard_normal(pred.shape).astype(np.float32)
    loss, tms, dpred = ctx.closure_loss(torch.tensor(target))
    ref_loss, ref_tms, ref_d = cnn.mse_loss(pred, target)
    assert abs(loss - ref_loss) < 1e-6 * ref_loss
    assert abs(tms - ref_tms) < 1e-12 * ref_tms
    assert rel_l2(dpred.cpu().numpy(), ref_d) < 1e-6
    # read=False leaves the means on the device and still writes the gradient
    d2 = torch.zeros_like(dpred)
    assert ctx.closure_loss(torch.tensor(target), d2, read=False)[:2] == (None, None)
    assert torch.equal(d2, dpred)


def test_loss_and_symmetry_argument_errors():
    """pm_closure_loss before a forward pass is a call-order error; pm_cube_symmetry rejects a perm that is not a
    permutation of 0, 1, 2 and a flip outside 0..7, before touching the device arrays."""
    import ctypes as C

    from paper_2607_17929_amd import PMContext
    from paper_2607_17929_amd import _lib as L
    ctx = PMContext(16, 64, 160.0, physics="scalar", precision="fp32", closure=True)
    r = np.random.default_rng(2)
    ctx.init_particles(r.random((64, 3)), np.zeros((64, 3), dtype=np.float32), opm.Background(160.0).tau(0.1))
    ctx.closure_set_params(torch.tensor(_params(), dtype=torch.float32))
    with pytest.raises(L.PMError):
        ctx.closure_loss(torch.zeros((64, 3)))
    lib = L.load()
    p = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    v = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    ptrs = [C.c_void_p(t.data_ptr()) for t in (p, v, v, p, v, v)]
    for perm, flip in [((0, 0, 1), 0), ((0, 1, 3), 0), ((2, 1, 0), 8), ((2, 1, 0), -1)]:
        assert lib.pm_cube_symmetry(ctx.ctx, 4, (C.c_int * 3)(*perm), flip, *ptrs) == L.PM_EINVAL
    assert lib.pm_cube_symmetry(ctx.ctx, 4, (C.c_int * 3)(2, 1, 0), 7, *ptrs) == L.PM_OK


def test_cube_symmetry_against_oracle():
    """pm_cube_symmetry for all 48 maps against the oracle's, bit for bit (including x = 0 and outputs that
    alias the inputs)."""
    import itertools
    from paper_2607_17929_amd import PMContext
    print("cube symmetry", flush=True)
    r = np.random.default_rng(12)
    m = 1000
    pos = r.random((m, 3))
    pos[0] = (0.0, 0.5, 0.999999)
    u = r.standard_normal((m, 3)).astype(np.float32)
    v = r.standard_normal((m, 3)).astype(np.float32)
    ctx = PMContext(16, 8, 160.0, physics="scalar", precision="fp32")
    tp, tu, tv = (torch.tensor(a, device="cuda") for a in (pos, u, v))
    for perm in itertools.permutations(range(3)):
        for flip in range(8):
            gp, gu, gv = ctx.cube_symmetry(tp, tu, tv, perm, flip)
            rp, ru, rv = cnn.cube_symmetry(pos, u, v, perm, flip)
            assert np.array_equal(gp.cpu().numpy(), rp) and np.array_equal(gu.cpu().numpy(), ru)
            assert np.array_equal(gv.cpu().numpy(), rv)
    ap, au, av = (t.clone() for t in (tp, tu, tv))
    ctx.cube_symmetry(ap, au, av, (2, 0, 1), 5, out=(ap, au, av))
    rp, ru, rv = cnn.cube_symmetry(pos, u, v, (2, 0, 1), 5)
    assert np.array_equal(ap.cpu().numpy(), rp) and np.array_equal(au.cpu().numpy(), ru)
    assert np.array_equal(av.cpu().numpy(), rv)


def test_closure_adam_step_parity():
    print("adam", flush=True)
    ctx, *_ = _setup()
    r = np.random.default_rng(9)
    p = r.standard_normal(cnn.N_PARAMS).astype(np.float32)
    m = (0.1 * r.standard_normal(cnn.N_PARAMS)).astype(np.float32)
    v = (0.01 * r.random(cnn.N_PARAMS)).astype(np.float32)
    g = r.standard_normal(cnn.N_PARAMS).astype(np.float32)
    tp, tm, tv, tg = (torch.tensor(a, device="cuda") for a in (p, m, v, g))
    ctx.closure_adam(tp, tm, tv, tg, 7, 1e-3)
    rp, rm, rv = cnn.adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64), g.astype(np.float64), 7,
                          lr=1e-3)
    assert rel_l2(tp.cpu().numpy(), rp) < 1e-6
    assert rel_l2(tm.cpu().numpy(), rm) < 1e-6 and rel_l2(tv.cpu().numpy(), rv) < 1e-6


def test_gather_grad_phi_matches_oracle():
    ctx, sim, n00, pos, n = _setup()
    g = ctx.gather_grad_phi().cpu().numpy()
    ref = opm.interpolate(opm.grad(sim.phi, n), pos, n).T
    assert rel_l2(g, ref) < 1e-10


def test_closure_training_beats_plain_force():
    """Small version of the closure experiment: 32^3 particles, 32^3 vs 64^3 meshes, 4 Mpc/h cells."""
    from paper_2607_17929_amd import closure
    print("closure training", flush=True)
    snaps, c1 = closure.make_pairs(seeds=[11, 12, 13], n_p=32 ** 3, n1=32, box=128.0, a_snaps=[0.2, 0.3, 0.4, 0.5],
                                   steps=40, spectrum=spectrum_power_law_m2)
    held, c1h = closure.make_pairs(seeds=[99], n_p=32 ** 3, n1=32, box=128.0, a_snaps=[0.3, 0.5], steps=40,
                                   spectrum=spectrum_power_law_m2)
    params, hist = closure.train(c1, snaps, closure.init_params(0), iters=400, lr=2e-3, log_every=100)
    plain, corr = closure.evaluate(c1h, held, params)
    print(f"held-out: plain 1x error {plain:.4e}, with closure {corr:.4e}", flush=True)
    assert np.mean(hist[-50:]) < np.mean(hist[:20])
    assert corr < 0.8 * plain


def test_parameters_from_host_memory_leave_the_run_untouched():
    """pm_closure_set_params from host memory stages the parameters inside the closure's own buffers:
    on a small run (100 particles, 16^3 mesh) the particles and fields are bit for bit what they were,
    and the network's output equals the one after binding the same parameters from device memory."""
    from paper_2607_17929_amd import PMContext
    print("closure parameters from host memory", flush=True)
    r = np.random.default_rng(21)
    pos = r.random((100, 3))
    u = 1e-3 * r.standard_normal((100, 3))
    ctx = PMContext(16, 100, 160.0, physics="scalar", precision="fp64", closure=True)
    ctx.init_particles(pos, u, opm.Background(160.0).tau(0.1))
    for _ in range(2):
        ctx.step(0.5)
    ctx.deposit()
    ctx.solve_metric(0.5)
    before = {k: ctx.get_field(k) for k in ("n00", "n0x", "nzz", "phi", "phi_prev", "chi")}
    pb, ub = ctx.get_particles()
    params = _params(4)
    ctx.closure_set_params(params, host=True)
    for k, v in before.items():
        assert np.array_equal(ctx.get_field(k), v), k
    pa, ua = ctx.get_particles()
    assert np.array_equal(pa, pb) and np.array_equal(ua, ub)
    ctx.closure_forward(False)
    out_host = ctx.closure_gather().cpu().numpy()
    ctx.closure_set_params(torch.tensor(params, dtype=torch.float32))
    ctx.closure_forward(False)
    assert np.array_equal(ctx.closure_gather().cpu().numpy(), out_host)
    ctx.update_particles(0.5)
    ctx.sync()


def test_reading_h_and_spectrum_between_solve_and_update():
    """With the closure on, reading h_ij or measuring P(k) between the solve and the update does not
    change the update: both use scratch that holds nothing between solves, not the deposit the closure
    reads its density feature from."""
    from paper_2607_17929_amd import PMContext
    print("h_ij and P(k) between solve and update", flush=True)
    pos, u, tau0, dtau = config_particles("zeldovich_32_scalar_fp64")
    params = _params(6)
    runs = []
    for probe in (False, True):
        ctx = PMContext(32, pos.shape[0], 320.0, physics="full", precision="fp64", closure=True)
        ctx.init_particles(pos, u, tau0)
        ctx.closure_set_params(torch.tensor(params, dtype=torch.float32))
        ctx.closure_enable(True)
        for i in range(3):
            ctx.deposit()
            ctx.solve_metric(dtau if i else 0.0)
            if probe:
                ctx.get_field("hxy")
                ctx.power_spectrum()
                ctx.get_field("hzz", device=True)
            ctx.update_particles(dtau)
        runs.append((ctx.get_particles()[0], gpu_fields_of(ctx)))
    (p0, f0), (p1, f1) = runs
    d = p1 - p0
    d -= np.round(d)
    assert np.max(np.abs(d)) * 32 < 1e-10
    for k in f0:
        assert rel_l2(f1[k], f0[k]) < 1e-12, k


def gpu_fields_of(ctx):
    return {k: ctx.get_field(k).astype(np.float64) for k in ("phi", "chi", "bx", "hxx")}

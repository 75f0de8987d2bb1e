"""GPU parity of the learned closure against its FP64 oracle (oracle/closure_oracle.py):
BF16-MFMA inference, FP32 training gradients and Adam steps, normalisation,
feature extraction, the Favre box filter, the eddy-viscosity targets, and the
fused stream-collide step with the closure.

Tolerances: inference is compared with the oracle's bf16-quantised forward
(same rounding of inputs, weights and hidden activations; the sums differ in
FP32 accumulation order, which can move a hidden activation by one bf16 ulp):
|nu_gpu - nu_ref| <= 2e-2 * rms(nu_ref) + 1e-6 per output.  Training runs in
FP32: gradients within 1e-4 of max |g_ref|, losses within 1e-5 relative.
FP64 filters and targets: 1e-12 relative (targets are stored as FP32: 1e-6).
"""
import numpy as np
import pytest

import oracle as O
from oracle import closure_oracle as C
from paper_2410_09739_amd import lbm as L
from paper_2410_09739_amd import workloads as W
from closure_checks import bf16_alternatives, explained_by_one_hidden_flip

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
W_ALPHA = O.feq(1.0, [0, 0, 0])


def _params(seed, bias=0.1):
    rng = np.random.default_rng(seed)
    p = C.init_params(seed)
    W1, b1, W2, b2, W3, b3 = C.unpack(p)
    b1 += bias * rng.standard_normal(64)
    b2 += bias * rng.standard_normal(64)
    b3 += bias * rng.standard_normal(6)
    return C.pack(W1, b1, W2, b2, W3, b3).astype(np.float32).astype(np.float64)


def _dev(a):
    """Device copy of a host array; the caller keeps the tensor alive while the
    library uses its pointer (the library runs on its own stream)."""
    t = torch.tensor(np.ascontiguousarray(a), device="cuda")
    torch.cuda.synchronize()
    return t


@pytest.mark.parametrize("n", [64, 1000, 4099, 1_000_003])
def test_mfma_inference_matches_bf16_oracle(n):
    p = _params(1)
    X = np.random.default_rng(2).standard_normal((n, 27)).astype(np.float32)
    xd = _dev(X)
    nud = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    L.lbm_closure_eval(p.astype(np.float32), xd.data_ptr(), nud.data_ptr(), n)
    got = nud.cpu().numpy().astype(np.float64)
    ref = C.forward_bf16(p, X.astype(np.float64))
    scale = np.sqrt(np.mean(ref ** 2))
    e = np.abs(got - ref)
    err = e.max()
    # The same bf16 roundings give the same network up to the order of the FP32
    # sums (~1e-7 relative); a hidden activation next to a bf16 rounding
    # boundary may round the other way on either side and move a node's outputs
    # by about one bf16 unit of that hidden unit times |W3| (measured: 1e-5 of
    # the rms at one of 4,099 nodes).  So 99 % of the outputs agree to the FP32
    # level (measured 1.2e-7 of the rms).
    q = np.quantile(e, [0.5, 0.9, 0.99]) / scale
    print(f"inference vs bf16 oracle / rms: median {q[0]:.1e}, 90% {q[1]:.1e}, 99% {q[2]:.1e}, max {err / scale:.1e}")
    assert q[2] <= 1e-6, q
    # Every node beyond the FP32 sums' reach (which tops out near 1e-5 of the
    # rms: 64-term sums of outputs up to several times the rms) is the oracle's
    # network with one hidden activation rounded to its other bf16 neighbour
    # (measured on 1,000,003 nodes: 947, all explained so).
    off = np.flatnonzero(np.any(e > 1e-5 * scale, axis=1))
    print(f"{off.size} of {n} nodes beyond the FP32 level")
    assert off.size <= 0.01 * n
    for i in off:
        assert explained_by_one_hidden_flip(p, X[i].astype(np.float64), got[i], 1e-5 * scale), i
    # and close to the exact network as well (BF16 quantisation only)
    exact, _ = C.forward(p, X)
    assert np.sqrt(np.mean((got - exact) ** 2)) <= 3e-2 * scale


@pytest.mark.parametrize("n", [1000, 2_000_003])  # not multiples of the 32-sample chunk; the second of
def test_mlp_loss_and_gradient_match_oracle(n):     # the size of a closure study's training set
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, 27)).astype(np.float32)
    Y = rng.standard_normal((n, 6)).astype(np.float32)
    p = _params(4)
    m = L.MLP(seed=0)
    m.set_params(p.astype(np.float32))
    m.set_normalisation(np.zeros(27), np.ones(27), 1.0)
    xd, yd = _dev(X), _dev(Y)
    loss, g = m.loss_grad(xd.data_ptr(), yd.data_ptr(), n)
    lref, gref = C.loss_and_grad(p, X.astype(np.float64), Y.astype(np.float64))
    assert loss == pytest.approx(lref, rel=1e-5)
    assert np.abs(g - gref).max() <= 1e-4 * np.abs(gref).max()
    m.close()


def test_mlp_normalisation_statistics_at_training_set_size():
    """Column means and standard deviations of 2,000,003 feature rows with a
    large common offset (the features' own scale: 1e-3 +- 3e-4), and the rms
    target scale, against numpy in FP64."""
    rng = np.random.default_rng(12)
    n = 2_000_003
    X = (3e-4 * rng.standard_normal((n, 27)) + 1e-3 * (1 + np.arange(27))).astype(np.float32)
    Y = (2e-3 * rng.standard_normal((n, 6))).astype(np.float32)
    xd, yd = _dev(X), _dev(Y)
    m = L.MLP(seed=0)
    m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), n)
    mu, sg, sy = m.get_normalisation()
    X64 = X.astype(np.float64)
    np.testing.assert_allclose(mu, X64.mean(0), rtol=1e-6)
    np.testing.assert_allclose(sg, X64.std(0), rtol=1e-5)
    assert sy == pytest.approx(np.sqrt(np.mean(Y.astype(np.float64) ** 2)), rel=1e-6)
    m.close()


def test_mlp_normalised_gradient_and_adam_steps_match_oracle():
    rng = np.random.default_rng(5)
    n = 777
    X = (3e-4 * rng.standard_normal((n, 27)) + 1e-3).astype(np.float32)
    Y = (2e-3 * np.abs(rng.standard_normal((n, 6)))).astype(np.float32)
    xd, yd = _dev(X), _dev(Y)
    m = L.MLP(seed=0)
    p0 = _params(6)
    m.set_params(p0.astype(np.float32))
    m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), n)
    mu, sg, sy = m.get_normalisation()
    np.testing.assert_allclose(mu, X.astype(np.float64).mean(0), rtol=1e-5, atol=1e-10)
    np.testing.assert_allclose(sg, X.astype(np.float64).std(0), rtol=1e-4)
    assert sy == pytest.approx(np.sqrt(np.mean(Y.astype(np.float64) ** 2)), rel=1e-5)
    Xs = (X.astype(np.float64) - mu) / sg
    Ys = Y.astype(np.float64) / sy
    # three Adam steps on sampled minibatches, replayed by the oracle
    batch, lr, seed = 96, 1e-3, 11
    hist = m.train(xd.data_ptr(), yd.data_ptr(), n, batch, 3, lr, seed)
    p, mm, vv = p0.copy(), np.zeros(C.NPARAM), np.zeros(C.NPARAM)
    for t in range(3):
        idx = C.sample_indices(seed, t, batch, n)
        lref, g = C.loss_and_grad(p, Xs[idx], Ys[idx])
        assert hist[t] == pytest.approx(lref, rel=1e-4)
        p, mm, vv = C.adam_step(p, g, mm, vv, t + 1, lr)
    got = m.get_params().astype(np.float64)
    # Adam moves every weight by about lr per step whatever the gradient size, so a
    # gradient entry near zero whose sign differs between FP32 and FP64 may move
    # one weight the other way: bound the fraction of such entries, not the max.
    d = np.abs(got - p)
    assert np.mean(d > 1e-5) < 2e-3 and d.max() <= 6 * lr
    # exported parameters act on raw features and return raw targets
    raw = m.export().astype(np.float64)
    ref_raw = C.fold_normalisation(got, mu.astype(np.float64), sg.astype(np.float64), sy)
    np.testing.assert_allclose(raw, ref_raw, rtol=1e-5, atol=1e-6 * np.abs(ref_raw).max())
    m.close()


def test_training_reduces_the_loss():
    rng = np.random.default_rng(7)
    n = 4096
    X = rng.standard_normal((n, 27)).astype(np.float32)
    Wt = rng.standard_normal((6, 27)) * 0.3
    Y = np.maximum(X @ Wt.T, 0.0).astype(np.float32)  # a learnable map
    m = L.MLP(seed=3)
    xd, yd = _dev(X), _dev(Y)
    m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), n)
    l0, _ = m.loss_grad(xd.data_ptr(), yd.data_ptr(), n)
    hist = m.train(xd.data_ptr(), yd.data_ptr(), n, 256, 300, 3e-3, 1)
    l1, _ = m.loss_grad(xd.data_ptr(), yd.data_ptr(), n)
    assert np.all(np.isfinite(hist))
    assert l1 < 0.1 * l0, (l0, l1)
    m.close()


def test_mlp_create_is_ordered_before_training():
    """lbm_mlp_create writes the initial parameters and clears the Adam moments
    on the object's own stream before it returns: work queued on the null stream
    at create changes nothing in what the training then computes."""
    rng = np.random.default_rng(17)
    n = 2048
    X = rng.standard_normal((n, 27)).astype(np.float32)
    Y = np.abs(rng.standard_normal((n, 6))).astype(np.float32)
    xd, yd = _dev(X), _dev(Y)
    out = []
    for busy in (False, True):
        if busy:
            big = torch.ones(1 << 27, device="cuda")
            for _ in range(100):
                big.mul_(1.0)
        m = L.MLP(seed=9)
        m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), n)
        m.train(xd.data_ptr(), yd.data_ptr(), n, 256, 5, 1e-3, 2)
        out.append(m.get_params())
        m.close()
        torch.cuda.synchronize()
    assert np.array_equal(out[0], out[1])


def _state(shape, seed, amp=0.05):
    nx, ny, nz = shape
    rho, u = W.random_fields(nx, ny, nz, seed=seed, u_amp=0.05)
    return O.init(rho, u) * W.random_factors((27, nz, ny, nx), seed=seed + 1, amplitude=amp)


@pytest.mark.parametrize("shape,storage", [((16, 12, 8), "f64"), ((136, 10, 6), "f32"), ((130, 8, 4), "f16dev")])
@pytest.mark.parametrize("walls", [False, True])
def test_coarsen_and_targets_match_oracle(walls, shape, storage):
    """Box filter, filtered strain and targets against the oracle on the
    GPU's own stored state (both sides in FP64 from the same populations):
    one segment, and rows of 3 segments with a ragged last one in FP32 and
    FP16 storage."""
    F = (2e-5, 0.0, 1e-5)
    g0 = _state(shape, 13)
    with L.Lattice(L.Config(*shape, storage=storage, walls_y=walls, nu=0.02, force=F)) as fine:
        fine.set_f(g0)
        fine.step(2)
        g = fine.get_f()
        nc = np.prod(shape) // 8
        rd = torch.zeros(nc, dtype=torch.float64, device="cuda")
        ud = torch.zeros(3 * nc, dtype=torch.float64, device="cuda")
        td = torch.zeros(6 * nc, dtype=torch.float64, device="cuda")
        sd = torch.zeros(6 * nc, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        L.lbm_coarsen(fine.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr())
        fine.synchronize()
    rho, u = O.macroscopic(g, F)
    rb, ut, tau = C.box_filter(rho, u)
    sbar = C.filtered_strain(rho, u, walls)
    cshape = (shape[0] // 2, shape[1] // 2, shape[2] // 2)
    np.testing.assert_allclose(rd.cpu().numpy().reshape(rb.shape), rb, rtol=1e-13)
    np.testing.assert_allclose(ud.cpu().numpy().reshape(ut.shape), ut, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(td.cpu().numpy().reshape(tau.shape), tau, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(sd.cpu().numpy().reshape(sbar.shape), sbar, rtol=1e-10,
                               atol=1e-12 * np.abs(sbar).max())
    nu_c = 0.01
    with L.Lattice(L.Config(*cshape, storage="f64", walls_y=walls, nu=nu_c)) as coarse:
        yd = torch.zeros((nc, 6), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        L.lbm_closure_targets(coarse.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr(), 0.1,
                              yd.data_ptr())
    ref = C.targets(rb, tau, C.strain(ut, walls), sbar, nu_c, eps_rel=0.1)
    assert np.abs(ref[:3]).max() > 0
    got = np.moveaxis(yd.cpu().numpy().reshape(cshape[::-1] + (6,)), -1, 0)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max() + 1e-30)


def test_coarsen_full_size_sampled_blocks():
    """The box filter at the size the closure study runs it: the fine channel
    384 x 192 x 192 in FP32 storage onto 192 x 96 x 96.  At sampled coarse
    nodes (walls, row ends, random) the filtered density, Favre velocity and
    sub-filter stress equal the oracle's filter of the GPU's own eight fine
    populations, read back through lbm_get_f_nodes."""
    nx, ny, nz = 384, 192, 192
    ut, h = 0.0025, 96.0
    F = (ut * ut / h, 0.0, 0.0)
    rho0, u0 = W.channel_turbulent_start(nx, ny, nz, u_bulk=15.7 * ut, amp=0.3, seed=77)
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    nc = cx * cy * cz
    rng = np.random.default_rng(9)
    sel = np.unique(np.concatenate([
        rng.integers(0, nc, 2000),
        np.array([(z * cy + y) * cx + x for x in (0, 31, 32, cx - 1) for y in (0, cy - 1) for z in (0, cz - 1)]),
    ]))
    X, Y, Z = sel % cx, (sel // cx) % cy, sel // (cx * cy)
    m = sel.size
    # fine node of (k, j, i) in block b, laid out as a (2, 2, 2m) pseudo-lattice
    kk, jj, ii = np.meshgrid(np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    fine_idx = (((2 * Z[None, None, None] + kk[..., None]) * ny + 2 * Y[None, None, None] + jj[..., None]) * nx
                + 2 * X[None, None, None] + ii[..., None])  # [k, j, i, b]
    with L.Lattice(L.Config(nx, ny, nz, storage="f32", walls_y=True, nu=ut * h / 180.0, force=F)) as fine:
        fine.init(rho0, u0)
        del rho0, u0
        fine.step(3)
        g = fine.get_f_nodes(np.moveaxis(fine_idx, -1, 2).ravel())  # order [k, j, b, i]
        rd = torch.zeros(nc, dtype=torch.float64, device="cuda")
        ud = torch.zeros(3 * nc, dtype=torch.float64, device="cuda")
        td = torch.zeros(6 * nc, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        L.lbm_coarsen(fine.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr())
        fine.synchronize()
    gs = g.reshape(27, 2, 2, 2 * m)
    rho, u = O.macroscopic(gs, F)
    rb, utl, tau = C.box_filter(rho, u)
    got_r = rd.cpu().numpy()[sel]
    got_u = ud.cpu().numpy().reshape(3, nc)[:, sel]
    got_t = td.cpu().numpy().reshape(6, nc)[:, sel]
    np.testing.assert_allclose(got_r, rb.reshape(m), rtol=1e-13)
    np.testing.assert_allclose(got_u, utl.reshape(3, m), rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(got_t, tau.reshape(6, m), rtol=1e-9, atol=1e-15)
    assert np.abs(tau[3]).max() > 1e-8  # resolved velocity differences inside the blocks


def _oracle_pre_collision(g, F, walls):
    """Streamed populations, Step 7 fields and central moments about u (FP64)."""
    e, _, _ = O.lattice()
    f = O.stream(g, walls_y=walls)
    rho, u = O.macroscopic(f, F, post_collision=False)
    kap = C.central_moments(f, u, e)
    return f, rho, u, kap


@pytest.mark.parametrize("walls,shape", [(False, (64, 5, 4)), (True, (64, 5, 4)), (True, (320, 3, 2))])
def test_features_match_oracle(walls, shape):
    F = (1e-5, -2e-5, 0.0)
    g0 = _state(shape, 17)
    with L.Lattice(L.Config(*shape, storage="f64", walls_y=walls, nu=0.02, force=F)) as lat:
        lat.set_f(g0)
        xd = torch.zeros((np.prod(shape), 27), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        L.lbm_closure_features(lat.ctx, xd.data_ptr())
        lat.synchronize()
    _, rho, _, kap = _oracle_pre_collision(g0, F, walls)
    ref = C.features(kap, rho).reshape(-1, 27)
    got = xd.cpu().numpy().astype(np.float64)
    # per feature, relative to its own range (floored: x_001 is ~1e-16 when F_z = 0)
    scale = np.maximum(np.abs(ref).max(0), 1e-6 * np.abs(ref).max())
    assert np.max(np.abs(got - ref) / scale) <= 1e-6


# The bound is set by the closure's BF16 inference, not by the storage form: a
# hidden activation one bf16 ulp apart moves nu_t by ~1e-3 of itself, omega_j,eff
# by ~omega^2 * 3 dnu and the populations by that times the second-order
# non-equilibrium moments (~1e-3 here): well below 1e-6 w_alpha.
@pytest.mark.parametrize("storage,tol,shape,oh", [("f64", 1e-6, (64, 6, 3), 1.0), ("f32", 2e-6, (64, 6, 3), 1.0),
                                                  ("f64", 1e-6, (320, 3, 2), 1.0), ("f16dev", 2e-6, (64, 6, 3), 1.0),
                                                  ("bf16dev", 2e-6, (64, 6, 3), 1.0), ("f64", 1e-6, (64, 6, 3), 1.3),
                                                  ("f32", 2e-6, (128, 4, 3), 1.3)])
def test_fused_closure_step_matches_oracle(storage, tol, shape, oh):
    """One fused step with the closure: the oracle streams, computes features,
    evaluates the bf16-quantised network, sets omega_4..9 per node and collides
    (320 wide: five segments per row, the persistent loop's row mapping).  With
    the paper's rates the kernel takes the unit-rate form of orders 3-6; with
    higher-order rates of 1.3 the general collision."""
    F = (1e-5, 0.0, -1e-5)
    walls = True
    nu = 0.005
    g0 = _state(shape, 23, amp=0.02)
    p = _params(8, bias=0.0)
    W1, b1, W2, b2, W3, b3 = C.unpack(p)
    # make the network's outputs O(1e-2) so that the eddy viscosities matter
    p = C.pack(W1 * 20.0, b1, W2, b2, W3 * 0.01, b3 + 5e-3).astype(np.float32).astype(np.float64)
    with L.Lattice(L.Config(*shape, storage=storage, walls_y=walls, nu=nu, force=F, omega_higher=oh)) as lat:
        lat.set_f(g0)
        g0q = lat.get_f()  # the state as stored (rounded to the storage form)
        lat.step(0)
        L.lbm_set_closure(lat.ctx, p.astype(np.float32))
        lat.step(1)
        got = lat.get_f()
    f, rho, u, kap = _oracle_pre_collision(g0q, F, walls)
    X = C.features(kap, rho).reshape(-1, 27)
    nu_t = C.forward_bf16(p, X)
    om = O.omega_table(nu, omega_higher=oh)
    ff = f.reshape(27, -1)

    def collide_node_with(i, nut):
        w = om.copy()
        w[4:10] = C.closure_rates(nut[None], om)[0]
        return O.collide_node(ff[:, i], w, F)

    ref = np.stack([collide_node_with(i, nu_t[i]) for i in range(ff.shape[1])], axis=1)
    # 16-bit storage: one unit in the last place of the stored deviation on top
    # (the stored value is rounded once, stochastically, after the collision)
    ulp = {"f16dev": 2.0 ** -10, "bf16dev": 2.0 ** -7}.get(storage, 0.0)
    bound = tol * W_ALPHA[:, None] + ulp * np.abs(ref - W_ALPHA[:, None]).max()
    err = np.abs(got.reshape(27, -1) - ref)
    ok = np.all(err <= bound, axis=0)
    # A feature that lies next to a bf16 rounding boundary may be rounded the
    # other way by the kernel, whose features carry the rounding of their own
    # arithmetic: either rounding is then a correct input to the network, and
    # at such nodes the step must match the oracle's with one of them.  "Next
    # to": within two FP32 units in the last place (the fp32 value itself may
    # sit on a bf16 tie), or, for the FP32 arithmetic of the reduced forms,
    # within 1e-7 of the feature's range (FP32 moments of order-0.1 values).
    eps = 1e-13 if storage == "f64" else 1e-7
    xtol = np.maximum(eps * np.abs(X).max(0), 2.0 * np.spacing(np.abs(X).astype(np.float32)))
    alts = bf16_alternatives(X, np.where(X == 0.0, 0.0, xtol))
    g27 = got.reshape(27, -1)
    for i in np.flatnonzero(~ok):
        for Xi in alts.get(i, []):
            r = collide_node_with(i, C.forward_bf16(p, Xi[None])[0])
            if np.all(np.abs(g27[:, i] - r) <= bound[:, 0]):
                ok[i] = True
                break
    assert np.all(ok), (np.flatnonzero(~ok)[:10], float((err / bound).max()))
    assert len(alts) <= 0.05 * X.shape[0]  # near-boundary features are rare (measured: 0.2-2.6 %)
    assert np.any(np.clip(nu_t, 0, None) > 1e-3)  # the closure was active


@pytest.mark.parametrize("shape,storage", [((192, 96, 96), "f32"), ((192, 96, 96), "f16dev"),
                                           ((384, 192, 192), "bf16dev")])
def test_fused_closure_step_full_size_sampled_nodes(shape, storage):
    """The closure workloads at full size: the coarse channel 192 x 96 x 96
    (FP32 and FP16 deviation storage) and the channel 384 x 192 x 192 (BF16
    deviation storage, 72 segments per wavefront of the persistent loop), with
    the trained parameters kept in the repository, in the launch configuration
    the benchmark times.  After a few fused steps from a perturbed channel
    state, the next step at sampled nodes (walls, seams, interior) matches the
    oracle's stream, features, bf16 network, per-node rates and collision,
    evaluated from the GPU's own previous state as stored."""
    import os
    nx, ny, nz = shape
    ut, h = 0.0025, ny / 2.0
    nu = ut * h / 180.0
    F = (ut * ut / h, 0.0, 0.0)
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_09739_amd",
                        "data", "closure_channel_192x96x96.npy")
    p = np.load(path).astype(np.float64)
    rho, u = W.channel_turbulent_start(nx, ny, nz, u_bulk=15.7 * ut, amp=0.3, seed=1234)
    rng = np.random.default_rng(5)
    sel = np.unique(np.concatenate([
        rng.integers(0, nx * ny * nz, 1500),
        np.array([(z * ny + y) * nx + x for x in (0, 1, 63, 64, nx - 1) for y in (0, 1, ny - 1) for z in (0, nz - 1)]),
    ]))
    with L.Lattice(L.Config(nx, ny, nz, storage=storage, walls_y=True, nu=nu, force=F)) as lat:
        lat.init(rho, u)
        L.lbm_set_closure(lat.ctx, p.astype(np.float32))
        lat.step(4)
        g_prev = lat.get_f()
        lat.step(1)
        g_next = lat.get_f().reshape(27, -1)[:, sel]
    e, _, _ = O.lattice()
    f = O.stream(g_prev, walls_y=True).reshape(27, -1)[:, sel]
    r, v = O.macroscopic(f, F, post_collision=False)
    kap = C.central_moments(f, v, e)
    X = C.features(kap, r)
    nu_t = C.forward_bf16(p, X)
    om = O.omega_table(nu)

    def collide_with(nut):
        wf = C.closure_rates(nut, om)
        out = np.zeros_like(f)
        for i in range(f.shape[1]):
            w = om.copy()
            w[4:10] = wf[i]
            out[:, i] = O.collide_node(f[:, i], w, F)
        return out

    ref = collide_with(nu_t)
    # Bound: FP32 arithmetic, plus the inference tolerance of
    # test_mfma_inference_matches_bf16_oracle (2e-2 rms + 1e-6 per output: one
    # bf16 rounding of an input or hidden unit may fall the other way on the
    # GPU) carried through the collision, one output group at a time.
    delta = 2e-2 * np.sqrt(np.mean(nu_t ** 2, axis=0)) + 1e-6
    infer = np.zeros_like(ref)
    for j in range(6):
        dev = np.zeros_like(ref)
        for sgn in (1.0, -1.0):
            nut = nu_t.copy()
            nut[:, j] += sgn * delta[j]
            dev = np.maximum(dev, np.abs(collide_with(nut) - ref))
        infer += dev
    # 16-bit storage: one unit in the last place of the stored deviation on top
    ulp = {"f16dev": 2.0 ** -10, "bf16dev": 2.0 ** -7}.get(storage, 0.0)
    base = 2e-6 * W_ALPHA[:, None] + ulp * np.abs(ref - W_ALPHA[:, None]).max()
    tol = base + infer
    err = np.abs(g_next - ref)
    assert np.all(err <= tol), float((err / tol).max())
    # most nodes see no rounding flip at all and sit at the arithmetic's level
    assert np.mean(np.all(err <= base, axis=0)) > 0.99
    assert np.clip(nu_t[:, :3], 0, None).max() > 1e-5  # the trained closure acts on the shear groups


def test_mlp_rejects_bad_arguments():
    """The training object's argument checks: empty sets, a batch or learning
    rate that is not positive, a non-positive target scale; the object then
    still trains."""
    n = 256
    xd = _dev(np.random.default_rng(1).standard_normal((n, 27)).astype(np.float32))
    yd = _dev(np.abs(np.random.default_rng(2).standard_normal((n, 6))).astype(np.float32))
    m = L.MLP(seed=4)
    bad = [lambda: m.loss_grad(xd.data_ptr(), yd.data_ptr(), 0),
           lambda: m.train(xd.data_ptr(), yd.data_ptr(), 0, 32, 5, 1e-3),
           lambda: m.train(xd.data_ptr(), yd.data_ptr(), n, 0, 5, 1e-3),
           lambda: m.train(xd.data_ptr(), yd.data_ptr(), n, 32, 5, 0.0),
           lambda: m.set_normalisation(np.zeros(27), np.ones(27), 0.0),
           lambda: m.set_normalisation(np.full(27, np.nan), np.ones(27), 1.0),
           lambda: m.set_normalisation(np.zeros(27), -np.ones(27), 1.0),
           lambda: m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), 0)]
    for call in bad:
        with pytest.raises(L.LBMError) as ei:
            call()
        assert ei.value.code == L.LBM_EINVAL
    m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), n)
    hist = m.train(xd.data_ptr(), yd.data_ptr(), n, 32, 5, 1e-3)
    assert np.all(np.isfinite(hist))
    m.close()


def test_set_closure_validates():
    with L.Lattice(L.Config(40, 4, 4, nu=0.02)) as lat:
        with pytest.raises(L.LBMError):
            L.lbm_set_closure(lat.ctx, np.zeros(C.NPARAM, np.float32))
    with L.Lattice(L.Config(64, 4, 4, nu=0.02)) as lat:
        bad = np.zeros(C.NPARAM, np.float32)
        bad[5] = np.nan
        with pytest.raises(L.LBMError):
            L.lbm_set_closure(lat.ctx, bad)
        L.lbm_set_closure(lat.ctx, np.zeros(C.NPARAM, np.float32))
        L.lbm_set_closure(lat.ctx, None)


def test_closure_pipeline_end_to_end():
    """Fine forced channel -> 2x2x2 filter -> coarse features and targets ->
    training on the GPU -> exported parameters drive a coarse run (acoustic
    scaling: nu_c = nu_f / 2, F_c = 2 F_f).  Checks the plumbing and that the
    trained closure changes the coarse run without destabilising it."""
    fine_shape = (128, 32, 32)
    nu_f, F_f = 0.01, 4e-6
    rho0, u0 = W.channel_turbulent_start(*fine_shape, u_bulk=0.03, amp=0.2, seed=3, kmax=2)
    with L.Lattice(L.Config(*fine_shape, storage="f32", walls_y=True, nu=nu_f, force=(F_f, 0, 0))) as fine:
        fine.init(rho0, u0)
        fine.step(300)
        nc = np.prod(fine_shape) // 8
        rd = torch.zeros(nc, dtype=torch.float64, device="cuda")
        ud = torch.zeros(3 * nc, dtype=torch.float64, device="cuda")
        td = torch.zeros(6 * nc, dtype=torch.float64, device="cuda")
        sd = torch.zeros(6 * nc, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        L.lbm_coarsen(fine.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr())
        fine.synchronize()
    cshape = tuple(s // 2 for s in fine_shape)
    ccfg = L.Config(*cshape, storage="f32", walls_y=True, nu=nu_f / 2, force=(2 * F_f, 0, 0))
    xd = torch.zeros((nc, 27), dtype=torch.float32, device="cuda")
    yd = torch.zeros((nc, 6), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with L.Lattice(ccfg) as coarse:
        L.lbm_init_device(coarse.ctx, rd.data_ptr(), ud.data_ptr())
        L.lbm_closure_features(coarse.ctx, xd.data_ptr())
        L.lbm_closure_targets(coarse.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr(), 0.1,
                              yd.data_ptr())
        coarse.synchronize()
    y = yd.cpu().numpy()
    assert np.all(np.isfinite(xd.cpu().numpy())) and np.all(y >= 0) and y[:, :3].max() > 0
    assert np.all(y[:, 3:] == 0)
    m = L.MLP(seed=1)
    m.fit_normalisation(xd.data_ptr(), yd.data_ptr(), nc)
    l0, _ = m.loss_grad(xd.data_ptr(), yd.data_ptr(), nc)
    hist = m.train(xd.data_ptr(), yd.data_ptr(), nc, 512, 400, 2e-3, 7)
    l1, _ = m.loss_grad(xd.data_ptr(), yd.data_ptr(), nc)
    assert np.all(np.isfinite(hist)) and l1 < 0.8 * l0, (l0, l1)
    params = m.export()
    m.close()
    results = {}
    for use in (False, True):
        with L.Lattice(ccfg) as coarse:
            L.lbm_init_device(coarse.ctx, rd.data_ptr(), ud.data_ptr())
            if use:
                L.lbm_set_closure(coarse.ctx, params)
            coarse.step(200)
            d = coarse.diagnostics()
            results[use] = (d, coarse.moments()[1])
    assert results[True][0]["n_nonfinite"] == 0
    assert results[True][0]["mass"] == pytest.approx(results[False][0]["mass"], rel=1e-5)
    du = np.abs(results[True][1] - results[False][1]).max()
    assert du > 0.0  # the closure acts
    assert du < 0.5 * np.abs(results[False][1]).max()


def test_trained_closure_removes_subfilter_flux_error_on_a_held_out_snapshot():
    """What the trained network gains over the method without it, a priori:
    on a filtered snapshot that training never saw, the eddy viscosities the
    network predicts (BF16 matrix-core inference, clamped to [0, 1/3] as the
    fused step applies them) must remove at least half of the flux error that
    its targets remove.  The error of a coarse node, per off-diagonal group
    j (xy, xz, yz), is the filtered fine flux minus the coarse model flux,
    a_j - nu_t,j S_j with a_j = nu_j (Sbar_j - S_j) - tau_j / (2 rho~) (the
    sub-filter stress tau, the Favre-filtered fine strain Sbar and the coarse
    strain S of the filtered velocity, here from the oracle's stencil); summed
    squares over the snapshot.  Without the network nu_t = 0.  (The a-posteriori
    gain on the mean profile of coarse channel runs is measured separately and
    is not reliable at these sizes.)"""
    fine_shape = (128, 64, 64)
    h, ut = 32.0, 0.0025
    nu_f, F_f = ut * h / 180.0, ut * ut / h
    nc = np.prod(fine_shape) // 8
    cshape = tuple(s // 2 for s in fine_shape)
    ccfg = L.Config(*cshape, storage="f32", walls_y=True, nu=nu_f / 2, force=(2 * F_f, 0, 0))
    rho0, u0 = W.channel_turbulent_start(*fine_shape, u_bulk=15.7 * ut, amp=0.3, seed=3)
    snaps = []
    with L.Lattice(L.Config(*fine_shape, storage="f32", walls_y=True, nu=nu_f, force=(F_f, 0, 0))) as fine, \
            L.Lattice(ccfg) as feat:
        fine.init(rho0, u0)
        fine.step(3000)
        for k in range(5):
            fine.step(1000)
            rd, ud = torch.zeros(nc, dtype=torch.float64, device="cuda"), torch.zeros(3 * nc, dtype=torch.float64,
                                                                                     device="cuda")
            td, sd = torch.zeros(6 * nc, dtype=torch.float64, device="cuda"), torch.zeros(6 * nc, dtype=torch.float64,
                                                                                         device="cuda")
            xd = torch.zeros((nc, 27), dtype=torch.float32, device="cuda")
            yd = torch.zeros((nc, 6), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            L.lbm_coarsen(fine.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr())
            fine.synchronize()
            L.lbm_init_device(feat.ctx, rd.data_ptr(), ud.data_ptr())
            L.lbm_closure_features(feat.ctx, xd.data_ptr())
            L.lbm_closure_targets(feat.ctx, rd.data_ptr(), ud.data_ptr(), td.data_ptr(), sd.data_ptr(), 0.1,
                                  yd.data_ptr())
            feat.synchronize()
            snaps.append((rd, ud, td, sd, xd, yd))
    X = torch.cat([s[4] for s in snaps[:-1]])
    Y = torch.cat([s[5] for s in snaps[:-1]])
    torch.cuda.synchronize()
    m = L.MLP(seed=2)
    m.fit_normalisation(X.data_ptr(), Y.data_ptr(), X.shape[0])
    m.train(X.data_ptr(), Y.data_ptr(), X.shape[0], 4096, 4000, 1e-3, 9)
    params = m.export()
    m.close()
    rd, ud, td, sd, xd, yd = snaps[-1]
    nud = torch.zeros((nc, 6), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    L.lbm_closure_eval(params, xd.data_ptr(), nud.data_ptr(), nc)
    torch.cuda.synchronize()
    nz, ny, nx = cshape[2], cshape[1], cshape[0]
    rho = rd.cpu().numpy().reshape(nz, ny, nx)
    u = ud.cpu().numpy().reshape(3, nz, ny, nx)
    tau = C.group(td.cpu().numpy().reshape(6, nz, ny, nx))[:3]
    sbar = C.group(sd.cpu().numpy().reshape(6, nz, ny, nx))[:3]
    S = C.group(C.strain(u, True))[:3]
    nu_c = nu_f / 2
    a = nu_c * (sbar - S) - tau / (2.0 * rho[None])

    def err(nu_t):  # nu_t [3, nz, ny, nx]
        return float(np.sum((a - nu_t * S) ** 2))

    def field(v):  # [nc, 6] -> the three off-diagonal groups as [3, nz, ny, nx]
        return np.moveaxis(v[:, :3].reshape(nz, ny, nx, 3), -1, 0).astype(np.float64)

    e0 = err(np.zeros_like(S))
    e_target = err(field(yd.cpu().numpy()))
    e_net = err(np.clip(field(nud.cpu().numpy()), 0.0, 1.0 / 3.0))
    print(f"held-out flux error: none {e0:.4e}, targets {e_target:.4e} ({1 - e_target / e0:.3%} less), "
          f"network {e_net:.4e} ({1 - e_net / e0:.3%} less)")
    assert e_target < e0
    assert e0 - e_net >= 0.5 * (e0 - e_target), (e0, e_target, e_net)


def test_refined_closure_lowers_the_mean_profile_error_on_a_held_out_start(tmp_path):
    """What the trained network gains, a posteriori.  The network kept in the
    repository was trained on a turbulent channel started from one random
    perturbation (seed 1234): a-priori targets from the filtered fine run, then
    one pass of mean-momentum-balance targets for the x-y shear group from its
    own coarse run, and an output gain that gives that coarse run the filtered
    fine bulk velocity (the closure study's --refine 1 --calibrate).  Here it
    runs on a channel it has never seen (seed 4321): fine 256 x 128 x 128 at
    Re_tau = 180 for 12 T*, coarse 128 x 64 x 64 in FP16 deviation storage for
    40 T* with statistics over the last 32, plain and with the fused closure,
    both against the box-filtered fine run.  Measured in the study: U(y)
    relative L2 error 0.134 (plain) and 0.020 (closure), bulk velocity 18.17 and
    15.94 u_tau against 16.06, rms error of u 0.130 and 0.100; those of v and w
    0.100/0.090 and 0.125/0.106 (printed, not asserted)."""
    import os
    from paper_2410_09739_amd.experiments import closure_channel as CC
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_09739_amd",
                        "data", "closure_channel_128x64x64_refined.npy")
    out = CC.main(["--shape", "256,128,128", "--tstar-transient", "6", "--tstar-stats", "6", "--coarse-run", "40",
                   "--coarse-stats", "32", "--gains", "1", "--load-params", path, "--coarse-storage", "f16dev",
                   "--flow-seed", "4321", "--save-params", str(tmp_path / "p.npy")])
    plain, cl = out["coarse"]["plain"], out["coarse"]["closure_s0_g1"]
    ub_f = out["fine"]["u_bulk_over_u_tau"]
    print(f"U(y) error: plain {plain['rel_l2_U_vs_filtered_fine']:.4f}, closure {cl['rel_l2_U_vs_filtered_fine']:.4f}; "
          f"U_b/u_tau: fine {ub_f:.3f}, plain {plain['u_bulk_over_u_tau']:.3f}, closure {cl['u_bulk_over_u_tau']:.3f}; "
          f"rms errors plain {[round(plain[f'rel_l2_{q}_rms_vs_filtered_fine'], 3) for q in 'uvw']}, "
          f"closure {[round(cl[f'rel_l2_{q}_rms_vs_filtered_fine'], 3) for q in 'uvw']}")
    assert cl["rel_l2_U_vs_filtered_fine"] <= 0.4 * plain["rel_l2_U_vs_filtered_fine"]
    assert abs(cl["u_bulk_over_u_tau"] - ub_f) < abs(plain["u_bulk_over_u_tau"] - ub_f)
    assert cl["rel_l2_u_rms_vs_filtered_fine"] <= 1.1 * plain["rel_l2_u_rms_vs_filtered_fine"]

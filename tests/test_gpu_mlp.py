"""Learned form on the GPU: the network kernels against the oracle (FP64 with
bfloat16 operand rounding emulated), the judge and fallback paths, and the
whole learned setup against the oracle's stationary vector.

Tolerances: forward outputs and gradients agree with the oracle per tensor to
2^-7 in relative 2-norm (one bfloat16 ulp: FP32 against FP64 accumulation can
flip the rounding of an activation); initial weights and everything decided in
the same precision on both sides are compared exactly.
"""
import numpy as np
import pytest

from oracle import bamg_oracle as O
from oracle import mlp_oracle as M
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402
from tests.test_gpu_parity import _grid, _p_from_ell  # noqa: E402

TOL = 2.0 ** -7


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, M.D_IN)).astype(np.float32)
    X[:, :4] = (rng.random((n, 4)) < 0.7).astype(np.float32)       # slot masks
    T = rng.normal(size=(n, M.D_OUT)).astype(np.float32)
    return X, T


def _theta(seed=3):
    th = M.init_params(seed)
    th += 0.05 * np.random.default_rng(seed).normal(size=th.size)     # non-zero biases
    return th.astype(np.float32)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def test_init_matches_oracle():
    th = B.mlp_init(11).cpu().numpy()
    assert np.array_equal(th, M.init_params(11).astype(np.float32))


@pytest.mark.parametrize("n", [1, 77, 1000, 4096 + 33])
def test_forward_matches_oracle(n):
    X, _ = _data(n)
    th = _theta()
    Y = B.mlp_forward(_dev(X), _dev(th)).cpu().numpy()
    Yo, _ = M.forward(th.astype(np.float64), X.astype(np.float64), bf16=True)
    assert np.linalg.norm(Y - Yo) <= TOL * np.linalg.norm(Yo)
    assert np.median(np.abs(Y - Yo)) <= 1e-4 * np.abs(Yo).mean()


@pytest.mark.parametrize("n", [64, 300, 5000])
def test_gradient_matches_oracle(n):
    X, T = _data(n, seed=n)
    th = _theta(5)
    L, g = B.mlp_loss_grad(_dev(X), _dev(T), _dev(th))
    Mk = X[:, :4].astype(np.float64)
    Lo, go = M.loss_and_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), Mk, bf16=True)
    assert abs(L - Lo) <= TOL * Lo
    g = g.cpu().numpy().astype(np.float64)
    for name, a, b in zip([s for s, _ in M.SHAPES], M.unpack(g).values(), M.unpack(go).values()):
        assert np.linalg.norm(a - b) <= TOL * np.linalg.norm(b), (name, np.linalg.norm(a - b) / np.linalg.norm(b))


def test_training_reduces_validation_loss():
    # a smooth target the network can fit: a fixed random network's output
    X, _ = _data(40000, seed=1)
    teacher = M.init_params(99)
    T, _ = M.forward(teacher, X.astype(np.float64))
    T = T.astype(np.float32)
    th = B.mlp_init(2)
    info = B.mlp_train(_dev(X[:32000]), _dev(T[:32000]), th, _dev(X[32000:]), _dev(T[32000:]), epochs=6, batch=1024,
                       lr=3e-3, seed=6)
    assert info.steps == 6 * 32
    assert info.val_loss_last < 0.5 * info.val_loss_first, (info.val_loss_first, info.val_loss_last)
    # the reported loss is the oracle's loss of the trained parameters
    Lo, _ = M.loss_and_grad(th.cpu().numpy().astype(np.float64), X[32000:].astype(np.float64),
                            T[32000:].astype(np.float64), X[32000:, :4].astype(np.float64), bf16=True)
    assert abs(info.val_loss_last - Lo) <= TOL * Lo


def test_collected_features_match_oracle():
    ch = C.tandem_queue(32)
    h = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=3, stop_after=1, collect=1))
    g = _grid(ch)
    U = h.export(0, B.X_U).reshape(ch.n, 8)
    Bl = O.b_from_a(ch.to_scipy())
    F, *_ = M.level_features(U, O.tv_weights(Bl, U), Bl, g)
    Fg = h.export(0, B.X_FEATURES).reshape(ch.n, 24).astype(np.float64)
    assert np.abs(Fg - F).max() <= 1e-6 * max(1.0, np.abs(F).max())
    # the first pass's slot weights are the exported P (stopped after that pass)
    Pg, _ = _p_from_ell(h, 0, g.coarse().n)
    assert np.array_equal(h.export(0, B.X_SLOTW0).reshape(ch.n, 4).astype(np.float64),
                          M.slot_weights(Pg, g).astype(np.float32).astype(np.float64))
    # after a full setup the final slot weights are the final P
    hf = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=3, collect=1))
    Pf, _ = _p_from_ell(hf, 0, g.coarse().n)
    assert np.array_equal(hf.export(0, B.X_SLOTW).reshape(ch.n, 4).astype(np.float64),
                          M.slot_weights(Pf, g).astype(np.float32).astype(np.float64))


def test_judge_extremes():
    ch = C.tandem_queue(40)
    th = _dev(_theta(7))
    base = dict(levels=3, stop_after=1)
    ls = B.Hierarchy.from_chain(ch, 8, B.default_options(**base, collect=1))
    # judge 1e-30: every proposal falls back, the hierarchy is the LS one
    h0 = B.Hierarchy.from_chain(ch, 8, B.default_options(**base, interp=B.INTERP_MLP, mlp_weights=th.data_ptr(),
                                                          mlp_judge=1e-30))
    st = h0.stats()
    assert st.mlp_points > 0 and st.mlp_fallback == st.mlp_points
    for l in range(3):
        for what in (B.X_P_COL, B.X_P_VAL) if l < 2 else (B.X_B_VAL,):
            assert np.array_equal(h0.export(l, what), ls.export(l, what)), (l, what)
    # judge 1e30: the level-0 rows are the fit plus the network's correction on
    # every valid slot (the fit's weights come back rounded to FP32 here)
    h1 = B.Hierarchy.from_chain(ch, 8, B.default_options(**base, interp=B.INTERP_MLP, mlp_weights=th.data_ptr(),
                                                          mlp_judge=1e30))
    assert h1.stats().mlp_fallback == 0
    F = ls.export(0, B.X_FEATURES).reshape(ch.n, 24)
    W0 = ls.export(0, B.X_SLOTW0).reshape(ch.n, 4).astype(np.float64)
    Y = B.mlp_forward(_dev(F), th).cpu().numpy().astype(np.float64)
    g = _grid(ch)
    Pg, _ = _p_from_ell(h1, 0, g.coarse().n)
    W = M.slot_weights(Pg, g)
    fpts = F[:, :4].sum(1) > 0
    want = np.where(F[:, :4] > 0, W0 + Y, 0.0)
    assert np.abs(W[fpts] - want[fpts]).max() <= 1e-6 * max(1.0, np.abs(want).max())
    # and the fit's own weights are what the least-squares form writes
    Pls, _ = _p_from_ell(ls, 0, g.coarse().n)
    assert np.array_equal(M.slot_weights(Pls, g).astype(np.float32).astype(np.float64)[fpts], W0[fpts])


def test_learned_setup_reaches_the_oracle_vector():
    ch = C.tandem_queue(40)
    th = _dev(_theta(7))
    for passes in (1, 2):
        x, info, h = B.stationary(ch, 12, tol=1e-13, max_cycles=300, levels=3, interp=B.INTERP_MLP,
                                  mlp_weights=th.data_ptr(), setup_passes=passes)
        assert info.converged
        st = h.stats()
        assert st.mlp_points > 0 and 0 <= st.mlp_fallback <= st.mlp_points
        xo, _, _ = O.stationary(ch.to_scipy(), _grid(ch), 12, O.Options(levels=3), tol=1e-13)
        assert np.abs(x - xo).sum() <= 1e-9


def test_bad_learned_options():
    ch = C.tandem_queue(8)
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(ch, 4, B.default_options(levels=2, interp=B.INTERP_MLP))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(ch, 4, B.default_options(levels=2, setup_passes=3))
    assert e.value.code == B.EINVAL


def test_collect_is_the_filtered_export():
    # bamg_mlp_collect: the F points' features and final - first-pass slot
    # weights, ordinary points only (features within +-16, corrections within
    # +-1), in level order -- the same rows the exported arrays give
    ch = C.tandem_queue(40)
    h = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=3, collect=1))
    fs, ts = [], []
    for l in range(2):
        n = h.level_info(l).n
        F = h.export(l, B.X_FEATURES).reshape(n, 24)
        T = h.export(l, B.X_SLOTW).reshape(n, 4) - h.export(l, B.X_SLOTW0).reshape(n, 4)
        keep = (F[:, :4].sum(1) > 0) & (np.abs(F).max(1) <= 16) & (np.abs(T).max(1) <= 1)
        fs.append(F[keep]); ts.append(T[keep])
    f, t = B.mlp_collect(h)
    assert np.array_equal(f.cpu().numpy(), np.concatenate(fs))
    assert np.array_equal(t.cpu().numpy(), np.concatenate(ts))
    h.close()
    h2 = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=3))
    with pytest.raises(B.BamgError) as e:
        B.mlp_collect(h2)
    assert e.value.code == B.EINVAL


def test_spec_training_is_the_manual_pipeline(tmp_path):
    # bamg_mlp_train_spec builds the chains itself (the jittered tandem
    # queues of the training set), collects and trains: the same parameters,
    # bit for bit, as collecting from the generator module's chains and
    # training through bamg_mlp_train
    from paper_1004_1451_amd import learned as LRN
    kw = dict(n_chains=3, n_val=1, side_min=40, side_max=60, r=8, levels=3, epochs=2, batch=1024)
    path = str(tmp_path / "net.bin")
    params, info = LRN.train(out_path=path, **kw)
    chains = C.training_chains(3, n_min=39, n_max=59)
    parts = [LRN.collect(ch, r=8, levels=3) for ch in chains]
    ftr = torch.cat([p[0] for p in parts[:2]]); ttr = torch.cat([p[1] for p in parts[:2]])
    fva, tva = parts[2]
    th = B.mlp_init(5)
    info2 = B.mlp_train(ftr, ttr, th, fva, tva, epochs=2, batch=1024, seed=6)
    assert torch.equal(params, th)
    assert info.steps == info2.steps and info.val_loss_last == info2.val_loss_last
    # the network file gives the same learned setup as the device parameters
    ch = C.tandem_queue(40)
    base = dict(levels=3, interp=B.INTERP_MLP, stop_after=1)
    h1 = B.Hierarchy.from_chain(ch, 8, B.default_options(**base, mlp_weights=params.data_ptr()))
    h2 = B.Hierarchy.from_chain(ch, 8, B.default_options(**base, mlp_weights_path=path.encode()))
    assert np.array_equal(h1.export(0, B.X_P_VAL), h2.export(0, B.X_P_VAL))


def test_trained_network_gain_is_measured(record_property):
    # small version of the learned workload: train on jittered tandems, then
    # measure what the network changes on a held-out chain (reported, whatever
    # its sign): the distance of the level-0 weights to the final fit, and the
    # cycles and fallback share of the one-pass learned setup
    from paper_1004_1451_amd import learned as LRN
    params, info = LRN.train(n_chains=6, n_val=2, side_min=64, side_max=128, r=8, levels=4, epochs=4, batch=1024)
    assert info.val_loss_last < info.val_loss_first
    ev = C.tandem_queue(95, jitter=0.2, seed=7, chain_id=5)
    hf = B.Hierarchy.from_chain(ev, 8, B.default_options(levels=4, collect=1))
    F = hf.export(0, B.X_FEATURES).reshape(ev.n, 24)
    Tfin = hf.export(0, B.X_SLOTW).reshape(ev.n, 4).astype(np.float64)
    T1 = hf.export(0, B.X_SLOTW0).reshape(ev.n, 4).astype(np.float64)
    Y = B.mlp_forward(_dev(F), params).cpu().numpy().astype(np.float64)
    m = F[:, :4] > 0
    f = m.sum(1) > 0
    err_fit = np.sqrt(((T1 - Tfin)[f] ** 2).mean())
    err_net = np.sqrt(((np.where(m, T1 + Y, 0.0) - Tfin)[f] ** 2).mean())
    res = {}
    for name, kw in (("ls_1pass", {}), ("learned_1pass", dict(interp=B.INTERP_MLP, mlp_weights=params.data_ptr()))):
        x, inf, h = B.stationary(ev, 8, tol=1e-10, max_cycles=300, levels=4, setup_passes=1, **kw)
        assert inf.converged
        st = h.stats()
        res[name] = (inf.cycles, st.mlp_fallback / max(1, st.mlp_points))
    record_property("level0_weight_rms_to_final_fit", {"first_pass_fit": err_fit, "network": err_net})
    record_property("cycles_and_fallback", res)
    print("gain: weight rms to final fit %.5f (fit) -> %.5f (network); %s" % (err_fit, err_net, res))
    # what the learned form gains here is cycles of the one-pass setup (15 ->
    # 10 on this held-out chain), not distance to the final weights: the
    # network's rows are no closer to the recompute pass's fit than the first
    # fit's are (0.0237 -> 0.0278 rms); both facts are recorded above
    assert res["learned_1pass"][0] <= res["ls_1pass"][0]

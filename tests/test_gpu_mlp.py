"""GPU parity of the learned initializer's BF16 matrix-core MLP against the
oracle (FP64 products of the same BF16 operands).

Bars: BF16 conversions bit-exact where the value converted is the same on
both sides (weights, inputs); values the kernels round to BF16 after an FP32
computation within one BF16 step of the FP64 value; FP32 outputs within
1e-4 relative L2. Every input is seeded; nothing the GPU computes is fed to
the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

TOL = 1e-4
DEV = "cuda"
HALF_STEP = 2.0 ** -8  # BF16 rounding error bound relative to the value (half of a 2^-7 spacing)


@pytest.fixture(scope="module")
def fgs():
    import paper_2604_01844_amd as m
    m.lib()
    oracle.build(force=False)
    return m


def to_bits(x64):
    """BF16-representable float64 -> int16 bit patterns."""
    u = (np.asarray(x64, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return u.view(np.int16)


def from_bits(t):
    """int16 tensor of BF16 bit patterns -> float64 array."""
    u = t.detach().cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def within_bf16(got, ref, floor):
    """Each value within BF16 rounding of the FP64 reference (plus a floor
    for the FP32 arithmetic before the rounding); <= 0 passes."""
    err = np.abs(got - ref)
    bound = HALF_STEP * np.abs(ref) + floor
    return float(np.max(err - bound))


def weights(seed):
    rng = np.random.default_rng(seed)
    return dict(w1=rng.normal(0, 0.05, (128, 544)).astype(np.float32), b1=rng.normal(0, 0.1, 128),
                w2=rng.normal(0, 0.12, (128, 128)).astype(np.float32), b2=rng.normal(0, 0.1, 128),
                w3=rng.normal(0, 0.12, (32, 128)).astype(np.float32), b3=rng.normal(0, 0.3, 32))


def inputs(n, seed):
    rows = (n + 31) // 32 * 32
    x = np.zeros((rows, 544))
    x[:n, :515] = oracle.mlp.bf16_round(si.normals((n, 515), seed))
    return x, rows


def oracle_weights(w):
    r = oracle.mlp.bf16_round
    return dict(w1=r(w["w1"]), b1=w["b1"].astype(np.float32).astype(np.float64), w2=r(w["w2"]),
                b2=w["b2"].astype(np.float32).astype(np.float64), w3=r(w["w3"]),
                b3=w["b3"].astype(np.float32).astype(np.float64))


def targets(n, seed):
    gs = si.gaussians(n, seed)
    return oracle.mlp.canonical_target(gs["density"].astype(np.float64), gs["log_scale"].astype(np.float64),
                                       gs["quat"].astype(np.float64))


def run_oracle(x, w, t, n):
    ow = oracle_weights(w)
    a = oracle.mlp.forward(x, ow["w1"], ow["b1"], ow["w2"], ow["b2"], ow["w3"], ow["b3"])
    rows = x.shape[0]
    tt = np.zeros((rows, 8))
    tt[:n] = t
    p, loss, g = oracle.mlp.heads(a["z3"][:n], t)
    dz3 = np.zeros((rows, 32))
    dz3[:n] = g
    grads = oracle.mlp.backward(x, a, ow["w2"], ow["w3"], dz3)
    return a, p, loss, g, grads


def test_pack_rounds_weights_bit_exactly(fgs):
    from paper_2604_01844_amd.mlp import InitMLP
    w = weights(1)
    net = InitMLP(w, DEV)
    torch.cuda.synchronize()
    for k, (wb, wbt) in enumerate(zip(net.wb, net.wbt)):
        ref = to_bits(oracle.mlp.bf16_round(w[f"w{k + 1}"]))
        np.testing.assert_array_equal(wb.cpu().numpy(), ref)
        np.testing.assert_array_equal(wbt.cpu().numpy(), ref.T)


@pytest.mark.parametrize("n", [1, 1001])
def test_gather_patches(fgs, n):
    from paper_2604_01844_amd.mlp import InitMLP
    nv = 48
    g = si.grid(nv)
    vol = np.abs(si.normals((nv, nv, nv), 5))
    mean = si.uniforms((3, n), 6) * 1.1 - 0.55  # some patches leave the grid, some means lie outside it
    mean = mean.astype(np.float32)
    extra = si.normals((3, n), 16)
    net = InitMLP(weights(1), DEV)
    vd = torch.from_numpy(vol).to(DEV)
    x, xt, rows = net.features(vd, fgs.Grid.from_dict(g), 1.7, torch.from_numpy(mean).to(DEV), transposed=True,
                               extra=torch.from_numpy(extra).to(DEV))
    torch.cuda.synchronize()
    got = from_bits(x)
    ref = oracle.mlp.patches(vol, g, mean.astype(np.float64), np.float64(np.float32(1.7)), extra=extra)
    assert within_bf16(got[:n], ref, 1e-6) <= 0
    assert np.all(got[n:] == 0)
    np.testing.assert_array_equal(xt.cpu().numpy(), x.cpu().numpy().T)
    # normalised by a device-side maximum (the library's own reduction)
    vmax = fgs.reduce_max(vd)
    assert float(vmax.item()) == float(vol.max())
    x2, _, _ = net.features(vd, fgs.Grid.from_dict(g), 1.0, torch.from_numpy(mean).to(DEV), norm_max=vmax)
    ref2 = oracle.mlp.patches(vol, g, mean.astype(np.float64), 1.0 / float(vol.max()))
    assert within_bf16(from_bits(x2)[:n], ref2, 1e-6) <= 0


@pytest.mark.parametrize("n", [1, 3001])
def test_forward(fgs, n):
    from paper_2604_01844_amd.mlp import InitMLP
    w = weights(2)
    x, rows = inputs(n, 7)
    net = InitMLP(w, DEV)
    acts = net.forward(torch.from_numpy(to_bits(x)).to(DEV), rows, keep_transposes=True)
    torch.cuda.synchronize()
    ref = run_oracle(x, w, targets(n, 8), n)[0]
    for k in ("z1", "z2", "z3"):
        assert oracle.rel_l2(acts[k].cpu().numpy(), ref[k]) <= TOL, k
    # the stored activations are the BF16 rounding of the kernel's own FP32
    # pre-activations (that decision is taken in FP32 on both sides)
    for k, z in (("h1", "z1"), ("h2", "z2")):
        got = from_bits(acts[k])
        zk = acts[z].cpu().numpy()
        np.testing.assert_array_equal(got, oracle.mlp.bf16_round(np.maximum(zk, 0)))
        np.testing.assert_array_equal(acts[k + "t"].cpu().numpy(), acts[k].cpu().numpy().T)


@pytest.mark.parametrize("n", [1, 3001])
def test_heads_and_loss(fgs, n):
    from paper_2604_01844_amd.mlp import InitMLP
    rows = (n + 31) // 32 * 32
    z3 = np.zeros((rows, 32), dtype=np.float32)
    z3[:n] = si.normals((n, 32), 9)
    t = targets(n, 10)
    t[::7, 0] = 0.0  # dead targets
    base = (si.normals(n, 18) * 0.5 - 4).astype(np.float32)
    net = InitMLP(weights(2), DEV)
    acts = {"z3": torch.from_numpy(z3).to(DEV)}
    bd = torch.from_numpy(base).to(DEV)
    p_inf, *_ = net.heads(acts, n, base_log_scale=bd)
    p, loss, dz3, dz3t = net.heads(acts, n, torch.from_numpy(t.astype(np.float32)).to(DEV), base_log_scale=bd)
    torch.cuda.synchronize()
    t32 = t.astype(np.float32).astype(np.float64)
    rp, rloss, rg = oracle.mlp.heads(z3[:n].astype(np.float64), t32, base.astype(np.float64))
    assert oracle.rel_l2(p.cpu().numpy(), rp) <= 1e-6
    np.testing.assert_array_equal(p.cpu().numpy(), p_inf.cpu().numpy())
    assert abs(float(loss.item()) - rloss) <= 1e-6 * abs(rloss)
    got = from_bits(dz3)
    assert within_bf16(got[:n], rg, 1e-6 * np.abs(rg).max()) <= 0
    assert np.all(got[n:] == 0)
    np.testing.assert_array_equal(dz3t.cpu().numpy(), dz3.cpu().numpy().T)


@pytest.mark.parametrize("n", [1, 3001, 65541])
def test_backward(fgs, n):
    from paper_2604_01844_amd.mlp import InitMLP
    w = weights(3)
    x, rows = inputs(n, 11)
    t = targets(n, 12)
    net = InitMLP(w, DEV)
    xb = torch.from_numpy(to_bits(x)).to(DEV)
    xt = xb.t().contiguous()
    acts = net.forward(xb, rows, keep_transposes=True)
    _, loss, dz3, dz3t = net.heads(acts, n, torch.from_numpy(t.astype(np.float32)).to(DEV))
    g = net.backward(xt, rows, acts, dz3, dz3t)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    # repeat: bit-identical (fixed-order split-K sums)
    g2 = net.backward(xt, rows, acts, dz3, dz3t)
    for k, v in g2.items():
        np.testing.assert_array_equal(v.cpu().numpy(), got[k])
    _, _, rloss, _, rgrads = run_oracle(x, w, t.astype(np.float32).astype(np.float64), n)
    assert abs(float(loss.item()) - rloss) <= 1e-4 * abs(rloss)
    for k in ("dw1", "db1", "dw2", "db2", "dw3", "db3"):
        assert oracle.rel_l2(got[k], rgrads[k]) <= TOL, (k, oracle.rel_l2(got[k], rgrads[k]))


def test_canonical_targets(fgs):
    from paper_2604_01844_amd.mlp import canonical_targets
    n = 5000
    gs = si.gaussians(n, 13)
    d = {k: torch.from_numpy(v).to(DEV) for k, v in gs.items()}
    got = canonical_targets(d["mean"], d["log_scale"], d["quat"], d["density"]).cpu().numpy().astype(np.float64)
    ref = oracle.mlp.canonical_target(gs["density"].astype(np.float64), gs["log_scale"].astype(np.float64),
                                      gs["quat"].astype(np.float64))
    np.testing.assert_array_equal(got[:, :4], ref[:, :4])  # density and sorted log-scales: exact
    # quaternions: equal up to FP32 rounding; sign fixed by w >= 0 except where w is ~0
    dot = np.abs(np.sum(got[:, 4:] * ref[:, 4:], axis=1))
    assert np.all(dot >= 1 - 1e-6)
    clear = np.abs(ref[:, 4]) > 1e-5
    assert np.max(np.abs(got[clear, 4:] - ref[clear, 4:])) <= 2e-6


def test_training_steps_reduce_the_loss(fgs):
    from paper_2604_01844_amd.mlp import InitMLP
    n = 2048
    nv = 48
    g = si.grid(nv)
    vol = np.abs(si.normals((nv, nv, nv), 14))
    mean = (si.uniforms((3, n), 15) * 0.8 - 0.4).astype(np.float32)
    t = targets(n, 16)
    net = InitMLP(InitMLP.init_weights(17), DEV)
    vd, md, td = torch.from_numpy(vol).to(DEV), torch.from_numpy(mean).to(DEV), \
        torch.from_numpy(t.astype(np.float32)).to(DEV)
    losses = [float(net.train_step(vd, fgs.Grid.from_dict(g), 1.0, md, td, 2e-3).item()) for _ in range(40)]
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0], losses

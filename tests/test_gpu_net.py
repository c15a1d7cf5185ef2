"""GPU start-field network (BF16 MFMA) against the FP64 oracle."""
import numpy as np
import pytest

from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _flat(params):
    return np.concatenate([p.ravel() for p in params]).astype(np.float32)


def _unflat(vec, C):
    shapes = [(C, 3, 3, 3), (C,), (C, C, 3, 3), (C,), (C, C, 3, 3), (C,), (2, C, 3, 3), (2,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(vec[o:o + k].reshape(s).astype(np.float64))
        o += k
    return out


def _problem(C, ny, nx, B, seed):
    from oracle import net
    rng = np.random.default_rng(seed)
    params = net.init_params(C, seed=seed)
    params[-1] = rng.standard_normal(2) * 0.1
    for i in (1, 3, 5):
        params[i] = rng.standard_normal(C) * 0.05
    Vext = rng.uniform(0.0, 2.0, (B, ny * nx))
    theta = rng.uniform(-np.pi, np.pi, (B, ny * nx))
    mu = 1.0
    x0 = np.stack([np.stack([Vext[b] - mu, np.cos(theta[b]), np.sin(theta[b])]).reshape(3, ny, nx)
                   for b in range(B)])
    target = rng.standard_normal((B, 2, ny, nx)) * 0.3
    return params, Vext, theta, mu, x0, target


@pytest.mark.parametrize("C,ny,nx,B", [(8, 8, 8, 2), (32, 16, 16, 3), (16, 12, 20, 1)])
def test_net_forward_matches_oracle(dev, C, ny, nx, B):
    import torch
    from oracle import net
    from paper_2310_03341_amd import api
    params, Vext, theta, mu, x0, _ = _problem(C, ny, nx, B, seed=C + ny)
    ref, _ = net.forward(params, x0)
    sn = api.StartNet(C, ny, nx, B, dev)
    assert sn.nparams == _flat(params).size
    sn.params.copy_(torch.from_numpy(_flat(params)))
    y = sn.forward(torch.from_numpy(Vext).to(dev), torch.from_numpy(theta).to(dev), mu)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(ref.shape)
    # BF16 activations and weights: relative error ~1e-2 of the output scale
    assert np.abs(got - ref).max() <= 3e-2 * max(1.0, np.abs(ref).max())


def _bf16(x):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _grads_bf16_model(params, x0, target):
    """The oracle's definitions evaluated on operands rounded where the kernels
    round them: BF16 input features, weights, stored activations and the
    data-gradient operand; weight and bias gradients from the unrounded output
    gradient.  The relu masks then come from the same BF16 activations."""
    from oracle import net
    h = _bf16(x0)
    acts = [h]
    for layer in range(4):
        z = net.conv(h, _bf16(params[2 * layer]), params[2 * layer + 1])
        h = _bf16(np.maximum(z, 0.0)) if layer < 3 else z
        acts.append(h)
    d = acts[-1] - target
    g = 2.0 * d / d.size
    grads = [None] * 8
    for layer in range(3, -1, -1):
        _, gW, gb = net.conv_backward(acts[layer], params[2 * layer], g)
        grads[2 * layer], grads[2 * layer + 1] = gW, gb
        if layer == 0:
            break
        gx, _, _ = net.conv_backward(acts[layer], _bf16(params[2 * layer]), _bf16(g))
        g = gx * (acts[layer] > 0.0)
    return grads


@pytest.mark.parametrize("seed", [5, 6])
def test_net_gradients_match_oracle(dev, seed):
    import torch
    from oracle import net
    from paper_2310_03341_amd import api
    C, ny, nx, B = 16, 12, 12, 2
    params, Vext, theta, mu, x0, target = _problem(C, ny, nx, B, seed=seed)
    loss_ref, grads_ref = net.loss_and_grads(params, x0, target)
    grads_bf = _grads_bf16_model(params, x0, target)
    sn = api.StartNet(C, ny, nx, B, dev)
    sn.params.copy_(torch.from_numpy(_flat(params)))
    loss = sn.backward(torch.from_numpy(Vext).to(dev), torch.from_numpy(theta).to(dev), mu,
                       torch.from_numpy(target.reshape(B, 2, -1).astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    assert abs(loss.item() - loss_ref) <= 2e-2 * loss_ref
    g = _unflat(sn.grads.cpu().numpy(), C)
    for i, (a, b, e) in enumerate(zip(g, grads_ref, grads_bf)):
        # against the same roundings: only FP32 accumulation order differs
        rel_bf = np.linalg.norm(a - e) / max(np.linalg.norm(e), 1e-12)
        assert rel_bf <= 5e-3, (i, rel_bf)
        # against FP64: the BF16 roundings themselves move the first layer's
        # gradient by 4-6 % (norm-wise) on these problems, later layers less
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 0.1, (i, rel)


def test_net_training_reduces_loss(dev):
    import torch
    from oracle import net
    from paper_2310_03341_amd import api
    C, ny, nx, B = 16, 12, 12, 4
    params, Vext, theta, mu, x0, _ = _problem(C, ny, nx, B, seed=9)
    # learnable target: a fixed smooth function of the inputs
    target = np.stack([0.5 * np.tanh(x0[:, 0]), 0.3 * (1 + x0[:, 1])], axis=1)
    sn = api.StartNet(C, ny, nx, B, dev)
    sn.params.copy_(torch.from_numpy(_flat(params)))
    Vd, Td = torch.from_numpy(Vext).to(dev), torch.from_numpy(theta).to(dev)
    tg = torch.from_numpy(target.reshape(B, 2, -1).astype(np.float32)).to(dev)
    l0 = sn.backward(Vd, Td, mu, tg).item()
    for _ in range(300):
        sn.backward(Vd, Td, mu, tg)
        sn.adam(3e-3)
    l1 = sn.backward(Vd, Td, mu, tg).item()
    assert l1 < 0.2 * l0, (l0, l1)


def test_adam_matches_oracle_elementwise(dev):
    """bdg_net_adam_step against Kingma & Ba's update in the oracle (FP64) over
    ten steps.  Gradients span 1e-9 .. 1, so that epsilon (1e-8) decides the
    smallest updates and its placement is checked too.  Tolerances: the kernel
    computes in FP32.  The first moment m_t = b1 m + (1 - b1) g sums terms of
    either sign, so its error is bounded by the terms' size, not by |m_t|:
    each step rounds three times and uses the FP32 constants b1 = fl(0.9) and
    fl(1 - fl(0.9)), which differ from 0.9 and 0.1 by the relative amounts
    d_b and d_c (d_c is about 4u: 1 - fl(0.9) is exact, fl(0.9) is not), so
    |err_t| <= b1 |err_{t-1}| + (3u + d_b + d_c) a_t with
    a_t = b1 a_{t-1} + (1 - b1)|g| and u = 2^-24, i.e.
    |err_t| <= t (3u + d_b + d_c) a_t.  The second moment sums positive terms (relative bound).  1 - 0.999f^t
    carries a relative error of about 1.3e-5 that the bias-corrected second
    moment only partly cancels."""
    import torch
    from oracle import net
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(41)
    nparam = 5000
    p0 = rng.standard_normal(nparam).astype(np.float32)
    scale = 10.0 ** rng.uniform(-9, 0, nparam)
    sn = api.StartNet(4, 4, 4, 1, dev)  # only its Adam state is used
    params = torch.from_numpy(p0).to(dev)
    grads = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ref_p, ref_m, ref_v = [p0.astype(np.float64)], [np.zeros(nparam)], [np.zeros(nparam)]
    a = np.zeros(nparam)  # running size of the first moment's terms
    u32 = 2.0 ** -24
    b1f = float(np.float32(0.9))
    d_b = abs(b1f - 0.9) / 0.9
    d_c = abs(float(np.float32(1.0) - np.float32(b1f)) - 0.1) / 0.1
    step_err = 3 * u32 + d_b + d_c
    lr = 1e-2
    for t in range(1, 11):
        g = (rng.standard_normal(nparam) * scale).astype(np.float32)
        grads.copy_(torch.from_numpy(g))
        api._call("bdg_net_adam_step", nparam, params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                  v.data_ptr(), t, float(lr), api._stream(dev))
        ref_p = net.adam_step(ref_p, [g.astype(np.float64)], ref_m, ref_v, t, lr=lr)
        a = 0.9 * a + 0.1 * np.abs(g.astype(np.float64))
        torch.cuda.synchronize()
        gp, gm, gv = params.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy()
        assert np.abs(gm - ref_m[0]).max() <= 1e-6 * np.abs(ref_m[0]).max()
        assert np.all(np.abs(gv - ref_v[0]) <= 3e-5 * ref_v[0] + 1e-38)
        assert np.all(np.abs(gm - ref_m[0]) <= t * step_err * a + 1e-45)
        # each step moves a parameter by at most ~lr; FP32 rounding of p itself
        assert np.all(np.abs(gp - ref_p[0]) <= 2e-5 * lr * t + 2e-7 * np.abs(ref_p[0])), t
    del sn


def test_start_fields_decode(dev):
    """bdg_net_start_fields: U = Vext + y[0], |Delta| = max(y[1], 0) of one sample."""
    import torch
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(3)
    C, ny, nx, B = 8, 10, 12, 3
    sn = api.StartNet(C, ny, nx, B, dev)
    y = torch.from_numpy(rng.standard_normal((B, 2, ny * nx)).astype(np.float32)).to(dev)
    Vext = rng.uniform(0, 2, ny * nx)
    U, D = sn.start_fields(y, 2, torch.from_numpy(Vext).to(dev))
    torch.cuda.synchronize()
    yh = y.cpu().numpy().astype(np.float64)
    assert np.array_equal(U.cpu().numpy(), Vext + yh[2, 0])
    assert np.array_equal(D.cpu().numpy(), np.maximum(yh[2, 1], 0.0))
    with pytest.raises(api.BdgError):
        sn.start_fields(y, 3, torch.from_numpy(Vext).to(dev))

"""The surrogate network's GPU kernels against the FP64 oracle network (oracle/mlp.py),
evaluated on the same bfloat16-rounded weights and layer inputs, and the surrogate
response inside the step against the exact integral."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ctx(nbox=1):
    from paper_1209_0461_amd import PMNu
    return PMNu(16, 8, 64.0, 8, 16, np.full(nbox, 0.3))


NIN, NPARAM = 16, 35329


def _unpack(blob):
    """Blob -> oracle params [(W (in, out), b)], feature mean/scale, target mean/scale."""
    o, params = 0, []
    for fi, fo in ((NIN, 128), (128, 128), (128, 128), (128, 1)):
        w = blob[o:o + fi * fo].astype(np.float64).reshape(fi, fo)
        o += fi * fo
        b = blob[o:o + fo].astype(np.float64)
        o += fo
        params.append((w, b))
    assert o == NPARAM
    mu, sg = blob[o:o + NIN].astype(np.float64), blob[o + NIN:o + 2 * NIN].astype(np.float64)
    ymu, ysg = float(blob[o + 4 * NIN]), float(blob[o + 4 * NIN + 1])
    return params, mu, sg, ymu, ysg


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, NIN)) * np.linspace(0.5, 2.0, NIN) + np.linspace(-1, 1, NIN)
    y = (np.sin(x[:, 0]) + 0.3 * x[:, 1] * x[:, 2] - 0.1 * x[:, 5] ** 2 + 0.05 * x[:, 10]
         + 0.2 * np.tanh(x[:, 15]))
    return x.astype(np.float32), y.astype(np.float32)


def _std_inputs(x, mu, sg):
    # the kernels standardise in FP32 before rounding to bfloat16
    return ((x.astype(np.float32) - mu.astype(np.float32)) / sg.astype(np.float32)).astype(np.float64)


def test_gradient_matches_oracle():
    import torch
    from paper_1209_0461_amd import binding
    from oracle import mlp
    ctx = _ctx()
    x, y = _data(200, 1)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    binding.pm_nu_surrogate_init(ctx.h, xd, yd, 123)
    blob = binding.pm_nu_surrogate_save(ctx.h)
    params, mu, sg, ymu, ysg = _unpack(blob)
    g = torch.zeros(NPARAM, device="cuda")
    loss = binding.pm_nu_surrogate_grad(ctx.h, xd, yd, g)
    xs = _std_inputs(x, mu, sg)
    ts = (y.astype(np.float64) - ymu) / ysg
    ref_loss, ref = mlp.mse_loss_and_grads(params, xs, ts, bf16=True)
    assert loss == pytest.approx(ref_loss, rel=2e-3)
    got = g.cpu().numpy().astype(np.float64)
    o = 0
    for li, (gw, gb) in enumerate(ref):
        for arr in (gw, gb):
            seg = got[o:o + arr.size].reshape(arr.shape)
            o += arr.size
            err = np.linalg.norm(seg - arr) / np.linalg.norm(arr)
            assert err < 1e-2, (li, arr.shape, err)
    ctx.close()


def test_gradient_after_training_steps_matches_oracle():
    """Also away from the initial weights (non-trivial GELU regime)."""
    import torch
    from paper_1209_0461_amd import binding
    from oracle import mlp
    ctx = _ctx()
    x, y = _data(4096, 2)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    binding.pm_nu_surrogate_init(ctx.h, xd, yd, 5)
    binding.pm_nu_surrogate_train(ctx.h, xd, yd, 3, 512, 3e-3, 9)
    params, mu, sg, ymu, ysg = _unpack(binding.pm_nu_surrogate_save(ctx.h))
    xs, ys = xd[:160], yd[:160]
    g = torch.zeros(NPARAM, device="cuda")
    binding.pm_nu_surrogate_grad(ctx.h, xs, ys, g)
    _, ref = mlp.mse_loss_and_grads(params, _std_inputs(x[:160], mu, sg),
                                    (y[:160].astype(np.float64) - ymu) / ysg, bf16=True)
    flat_ref = np.concatenate([a.reshape(-1) for pair in ref for a in pair])
    err = np.linalg.norm(g.cpu().numpy() - flat_ref) / np.linalg.norm(flat_ref)
    assert err < 1e-2
    ctx.close()


def test_predict_matches_oracle_forward():
    import torch
    from paper_1209_0461_amd import binding
    from oracle import mlp
    ctx = _ctx()
    x, y = _data(1000, 3)   # 1000 = ragged tail of 32-row tiles
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    binding.pm_nu_surrogate_init(ctx.h, xd, yd, 77)
    binding.pm_nu_surrogate_train(ctx.h, xd, yd, 2, 256, 3e-3, 1)
    params, mu, sg, ymu, ysg = _unpack(binding.pm_nu_surrogate_save(ctx.h))
    out = torch.empty(1000, device="cuda")
    binding.pm_nu_surrogate_predict(ctx.h, xd, out)
    ref, _ = mlp.forward(params, _std_inputs(x, mu, sg), bf16=True)
    ref = ref[:, 0] * ysg + ymu
    assert np.abs(out.cpu().numpy() - ref).max() < 5e-3 * ysg
    ctx.close()


def test_training_reduces_loss():
    import torch
    from paper_1209_0461_amd import binding
    ctx = _ctx()
    x, y = _data(16384, 4)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    binding.pm_nu_surrogate_init(ctx.h, xd, yd, 3)
    g = torch.zeros(NPARAM, device="cuda")
    l0 = binding.pm_nu_surrogate_grad(ctx.h, xd, yd, g)
    l1 = binding.pm_nu_surrogate_train(ctx.h, xd, yd, 30, 1024, 2e-3, 11)
    assert l1 < 0.05 * l0, (l0, l1)
    ctx.close()


def test_blob_roundtrip_and_bad_blob():
    import torch
    from paper_1209_0461_amd import binding, PMNuError
    ctx = _ctx()
    with pytest.raises(PMNuError) as e:   # nothing loaded yet
        binding.pm_nu_surrogate_save(ctx.h)
    assert e.value.code == -7
    x, y = _data(256, 5)
    binding.pm_nu_surrogate_init(ctx.h, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 1)
    blob = binding.pm_nu_surrogate_save(ctx.h)
    ctx2 = _ctx()
    binding.pm_nu_surrogate_load(ctx2.h, blob)
    assert np.array_equal(binding.pm_nu_surrogate_save(ctx2.h), blob)
    bad = blob.copy()
    bad[NPARAM + NIN] = 0.0     # zero feature scale
    with pytest.raises(PMNuError):
        binding.pm_nu_surrogate_load(ctx2.h, bad)
    ctx.close()
    ctx2.close()

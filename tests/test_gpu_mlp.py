"""GPU tests of the cost-model network kernels against the fp64 oracle, and
of training, persistence and use of the learned cost model."""
import os
import tempfile

import numpy as np
import pytest
import torch

from oracle import mlp as OM
from oracle import planner as OP
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

SIZES = [16, 64, 64, 64, 1]


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _u(seed, n, stream=0):
    return synth.splitmix64(seed, stream, 0, n).astype(np.float64) / 2.0 ** 63 - 1.0


def _params(seed):
    ps = OM.init_params(SIZES, _u(seed, 16 * 64 + 2 * 64 * 64 + 64))
    for i in range(1, len(ps), 2):
        ps[i] = 0.1 * _u(seed + i, ps[i].size, 1)
    flat = np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)
    assert flat.size == A.MLP_PARAMS
    # the oracle sees exactly the fp32 values the device sees
    at, out = 0, []
    for p in ps:
        out.append(flat[at:at + p.size].astype(np.float64).reshape(p.shape))
        at += p.size
    return flat, out


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B", [1, 7, 256, 1000])
def test_forward_backward_match_oracle(ctx, B):
    flat, ps = _params(3)
    x = _u(4, B * 16, 2).reshape(B, 16).astype(np.float32)
    y = _u(5, B, 3).astype(np.float32)
    dp = torch.from_numpy(flat).cuda()
    dx = torch.from_numpy(x).cuda()
    dt = torch.from_numpy(y).cuda()
    out = torch.empty(B, dtype=torch.float32, device="cuda")
    A.mlp_forward(ctx, dp, dx, out)
    grad = torch.empty(A.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    A.mlp_backward(ctx, dp, dx, dt, grad, loss)
    torch.cuda.synchronize()
    want, _ = OM.forward(ps, x.astype(np.float64))
    assert _rel(out.cpu().numpy(), want) <= 1e-5
    assert abs(loss.item() - OM.loss(ps, x.astype(np.float64), y.astype(np.float64))) <= \
        1e-5 * max(1.0, abs(loss.item()))
    g = grad.cpu().numpy()
    og = OM.backward(ps, x.astype(np.float64), y.astype(np.float64))
    at = 0
    for k, t in enumerate(og):
        e = _rel(g[at:at + t.size], t.reshape(-1))
        say("grad tensor", k, "rel err", e)
        assert e <= 1e-4, k
        at += t.size


def test_adam_step_matches_oracle(ctx):
    flat, ps = _params(6)
    g = (_u(7, A.MLP_PARAMS, 4) * 1e-2).astype(np.float32)
    m = (_u(8, A.MLP_PARAMS, 5) * 1e-3).astype(np.float32)
    v = np.abs(_u(9, A.MLP_PARAMS, 6) * 1e-4).astype(np.float32)
    dp, dg, dm, dv = (torch.from_numpy(a.copy()).cuda() for a in (flat, g, m, v))
    A.mlp_adam(ctx, dp, dg, dm, dv, 1e-3, 0.9, 0.999, 1e-8, 5)
    torch.cuda.synchronize()
    # oracle: same moments, step 5
    opt = OM.Adam([flat.astype(np.float64)], lr=1e-3)
    opt.m = [m.astype(np.float64)]
    opt.v = [v.astype(np.float64)]
    opt.t = 4
    p64 = [flat.astype(np.float64)]
    opt.step(p64, [g.astype(np.float64)])
    assert _rel(dp.cpu().numpy() - flat, p64[0] - flat) <= 1e-4
    assert _rel(dm.cpu().numpy(), opt.m[0]) <= 1e-6
    assert _rel(dv.cpu().numpy(), opt.v[0]) <= 1e-6


def test_train_save_load_predict_and_fallback(ctx):
    rep = A.costmodel_train(ctx, A.train_opts(n_samples=400, epochs=60, min_log2_n=12, max_log2_n=16, reps=2))
    say("train report", rep)
    assert rep["n_train"] + rep["n_val"] == 400 and np.isfinite(rep["val_loss"])
    n = 1 << 16
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    sec = A.Section.from_spec(st, synth.random_program(3, spec.n_fields)[2])
    lay = A.Layout.soa(st)
    p1 = A.costmodel_predict(ctx, sec, lay)
    assert p1 > 0
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        A.costmodel_save(ctx, path)
        ctx2 = A.Ctx(0)
        A.costmodel_load(ctx2, path)
        assert A.costmodel_predict(ctx2, sec, lay) == p1
        raw = bytearray(open(path, "rb").read())
        raw[100] ^= 0xFF
        open(path, "wb").write(bytes(raw))
        with pytest.raises(A.AdhaError) as e:
            A.costmodel_load(ctx2, path)
        assert e.value.status == A.ERR_IO
        with pytest.raises(A.AdhaError):
            A.costmodel_predict(ctx2, sec, lay)          # no model after a failed load
        prog = A.Program(st, [sec])
        pl = A.Plan.create(ctx2, prog, A.plan_opts(cost=A.COST_LEARNED, catalogue=A.CAT_AOS_SOA))
        assert pl.status == A.WARN_FALLBACK              # measured enumeration instead

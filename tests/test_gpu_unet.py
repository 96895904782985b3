"""The learned preconditioner: GPU forward and gradients against the float64
reference network, training on GPU, and its use inside the solver (where the
V-cycle stays the fallback and the true residual the judge)."""
import numpy as np
import pytest

import workloads as wl
import unet_reference as ref
from oracle.fv import assemble
from oracle.heads import heads_problem
from gpu_util import device_problem, check_heads, announce

pytestmark = pytest.mark.gpu


def _setup(lt, nx=128, ny=16, seed=5):
    import torch
    p = wl.make_problem("C4_train", n=(nx, ny), seed=seed)
    h = device_problem(lt, p)
    K, m = assemble(p.n, p.h, p.kappa, p.S)
    D = K.diagonal()
    return p, h, D, m


def _rand(nvec, N, seed):
    import torch
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nvec, 2, N))
    return a, torch.tensor(a, dtype=torch.float64, device="cuda").contiguous()


def test_forward_matches_reference(lt):
    import torch
    p, h, D, m = _setup(lt)
    announce("unet forward")
    net = lt.UNet(seed=3)
    params = net.get_params()
    tau = 2e5 + 7e5j
    rn, r = _rand(2, p.N, 1)
    e = torch.empty_like(r)
    lt.lt_unet_apply(net, h, tau, r, e, 2)
    got = e.cpu().numpy()
    want = ref.apply(params.astype(np.float64), rn, D, m, tau, p.n[0], p.n[1])
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("forward rel err", err, flush=True)
    assert err <= 5e-2  # BF16 activations and weights against float64
    net.close()
    h.close()


def test_gradient_matches_reference(lt):
    import torch
    p, h, D, m = _setup(lt)
    announce("unet gradient")
    net = lt.UNet(seed=4)
    params = net.get_params().astype(np.float64)
    # the GPU multiplies with BF16 copies of the convolution weights: compare
    # against the float64 reference at those rounded weights (the head stays FP32)
    pb = torch.tensor(params).to(torch.bfloat16).to(torch.float64).numpy()
    pb[-34:] = params[-34:]
    tau = 5e4 + 3e5j
    rn, r = _rand(2, p.N, 2)
    en, e = _rand(2, p.N, 3)
    g = lt.lt_unet_grad(net, h, tau, r, e, 2).astype(np.float64)
    _, gr = ref.loss_and_grad(pb, rn, en, D, m, tau, p.n[0], p.n[1])
    cos = g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print("grad cos", cos, "rel", rel, flush=True)
    # BF16 activations and BF16 pre-activation gradients bound the agreement
    assert cos >= 0.99 and rel <= 0.15
    # every layer's gradient, not just the large ones
    off = 0
    for ci, co in ref.LAYERS:
        n = 9 * ci * co + co
        a, b = g[off:off + n], gr[off:off + n]
        assert np.linalg.norm(a - b) <= 0.3 * np.linalg.norm(b) + 1e-12, (ci, co)
        assert a @ b >= 0.97 * np.linalg.norm(a) * np.linalg.norm(b), (ci, co)
        off += n
    net.close()
    h.close()


def test_training_reduces_loss_on_a_fixed_batch(lt):
    import torch
    from paper_1409_2556_amd.train_unet import make_batch
    p, h, D, m = _setup(lt, 128, 128, seed=10000)
    announce("unet overfit")
    rng = np.random.default_rng(0)
    tau = 1e5 + 4e5j
    r, e = make_batch(lt, h, p, 8, tau, rng)
    net = lt.UNet(seed=1)
    losses = [lt.lt_unet_train_step(net, h, tau, r, e, 8, 2e-3) for _ in range(60)]
    print("loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    net.close()
    h.close()


@pytest.mark.parametrize("kind", ["random", "nan", "zero"])
@pytest.mark.parametrize("prec", [0, 1])
def test_solver_with_network_still_matches_oracle(lt, kind, prec):
    p = wl.make_problem("C4_train", n=(128, 128), seed=10003, nsrc=2, nrec=6)
    announce("unet solver", kind, prec)
    h = device_problem(lt, p)
    net = lt.UNet(seed=2)
    if kind == "nan":
        w = net.get_params()
        w[::7] = np.nan
        net.set_params(w)
    elif kind == "zero":
        net.set_params(np.zeros(net.nparams, dtype=np.float32))
    lt.lt_unet_attach(h, net)
    tol = 1e-10 if prec == 0 else 1e-8
    o = lt.make_opts(tol=tol, precision=prec, precond=lt.LT_PRECOND_UNET_GMG)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    print(kind, prec, "net", st["net_applied"], st["net_rejected"], "vc", st["vcycles"], flush=True)
    assert st["rc"] == 0
    check_heads(phi.cpu().numpy(), heads_problem(p), 1e-6 if prec == 0 else 1e-5, f"unet {kind} prec {prec}")
    assert st["true_relres_max"] <= tol
    assert st["net_applied"] > 0
    if kind == "nan":
        assert st["net_rejected"] == st["net_applied"]
    lt.lt_unet_attach(h, None)
    net.close()
    h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_trained_network_in_the_solver_matches_oracle(lt, prec):
    """A network trained by the library's own kernels (400 Adam steps on 128x128 fields), kept
    on for every preconditioner solve of an unseen 256x256 field: the heads still match the
    direct-solve oracle element by element, since every guess is followed by the V-cycle
    refinement and the true residual judges the result."""
    from paper_1409_2556_amd.train_unet import train
    p = wl.make_problem("C4_256", nsrc=3, nrec=8)
    announce("trained unet solver", prec, p.n)
    net, hist = train(steps=400, batch=8, lr=1e-3, verbose=False)
    print("training loss (last 20)", float(np.mean(hist[-20:])), flush=True)
    assert np.mean(hist[-20:]) < np.mean(hist[:20])
    h = device_problem(lt, p)
    lt.lt_unet_attach(h, net)
    tol = 1e-10 if prec == 0 else 1e-8
    o = lt.make_opts(tol=tol, precision=prec, precond=lt.LT_PRECOND_UNET_GMG, net_keep=1e30)
    phi, st = lt.lt_solve(h, p.sources, p.q, p.times, p.nz_contour, p.receivers, o)
    print(prec, "net", st["net_applied"], st["net_rejected"], "disabled", st["net_disabled_at"], "iters",
          st["iters_max"], "vcycles", st["vcycles"], "true", st["true_relres_max"], flush=True)
    assert st["rc"] == 0
    assert st["net_disabled_at"] == 0 and st["net_applied"] >= st["iters_max"]
    check_heads(phi.cpu().numpy(), heads_problem(p, workers=8), 1e-6 if prec == 0 else 1e-5,
                f"trained unet prec {prec}")
    assert st["true_relres_max"] <= tol
    lt.lt_unet_attach(h, None)
    net.close()
    h.close()

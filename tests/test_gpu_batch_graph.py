"""Mixed-size frame batches captured into one HIP graph (via torch's graph
capture of the library's launches on the capturing stream): every replay
reproduces the eager results exactly, with eager work and synchronisation
between replays; and the FP32 blur's vector-ALU path (used for shapes the
matrix-core kernel is not instantiated for) matches Eq. (8)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
import synthetic  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_06713_amd as t
    return t


@pytest.fixture(scope="module")
def basis():
    A, _ = opsf.basis_draws(600, seed=31)
    return opsf.pca_basis(opsf.psf_batch(A, 64, 33), 100)[0]


def test_render_vector_alu_path(t):
    say("render fp32 vector path K=40")
    A, _ = opsf.basis_draws(300, seed=8)
    Psi = opsf.pca_basis(opsf.psf_batch(A, 64, 33), 40)[0]
    H, W, C = 30, 50, 2
    plan = t.Plan(H, W, C, 64, 64, basis=Psi)
    img = synthetic.test_image(C, H, W, 4, seed=3)[None]
    beta = synthetic.random_coefficients((1, H, W, 40), 0.05, 4)
    beta[..., 0] += 1.0
    out = torch.empty((1, C, H, W), dtype=torch.float32, device="cuda")
    plan.render(torch.tensor(img, device="cuda"), torch.tensor(beta, device="cuda"), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    for c in range(C):
        ref = orender.render_basis(img[0, c].astype(np.float64), beta[0].astype(np.float64), Psi, 33)
        assert np.linalg.norm(got[c] - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("learned", [False, True])
def test_mixed_size_batch_graph_replays_match_eager(t, basis, learned):
    say(f"graph batch learned={learned}")
    sizes = [(2, 64, 64, 128, 128), (2, 48, 96, 128, 256), (1, 96, 64, 256, 128)]
    dev = torch.device("cuda")
    plans, bufs = [], []
    net = None
    for (F, H, W, Gh, Gw) in sizes:
        kw = dict(basis=basis)
        if learned:
            kw.update(p2s_mode=t.P2S_LEARNED, precision=t.BF16)
        p = t.Plan(H, W, 3, Gh, Gw, **kw)
        if learned:
            if net is None:
                net = t.Mlp(p, batch=64, seed=4)
            t.plan_set_mlp(p, net)
        kb = 112 if learned else 100
        bt = torch.bfloat16 if learned else torch.float32
        img = torch.tensor(synthetic.test_image(3, H, W, 8, seed=F + H)[None].repeat(F, 0), device=dev)
        b = dict(img=img, zern=torch.empty((F, 35, H, W), device=dev),
                 beta=torch.empty((F, H, W, kb), dtype=bt, device=dev),
                 blur=torch.empty((F, 3, H, W), device=dev), out=torch.empty((F, 3, H, W), device=dev),
                 ws=p.workspace(F), dr=list(synthetic.d_over_r0_uniform(F, 1.0, 4.0, H)))
        plans.append(p)
        bufs.append(b)

    def run_all(frame0):
        for p, b in zip(plans, bufs):
            p.sample_zernike(b["dr"], 5, frame0, b["zern"], b["ws"])
            p.p2s(b["zern"], b["beta"], b["ws"])
            p.render(b["img"], b["beta"], b["blur"])
            p.warp(b["blur"], b["zern"], b["out"])

    run_all(0)
    torch.cuda.synchronize()
    eager = [b["out"].clone() for b in bufs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run_all(0)                      # warm the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        run_all(0)
    for rep in range(3):
        for b in bufs:
            b["out"].zero_()
        scratch = torch.randn(1 << 20, device=dev)   # eager work between replays
        (scratch * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for e, b in zip(eager, bufs):
            assert torch.equal(e, b["out"]), rep

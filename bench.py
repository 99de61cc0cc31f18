"""Benchmark of the dense-field phase-to-space renderer on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the plain FP32 form): 512 x 512 x 3 float32 frames, Noll modes
2..36 sampled on a 1024 x 1024 padded grid, exact pupil-FFT PSFs (64 x 64
pupil, 33 x 33 crop) projected on a K = 100 PCA basis, FP32 basis blur and
bilinear tilt warp, 16 independent frames per step with D/r0 cycling through
1, 2 and 4.  One step = sample -> P2S -> render -> warp for the 16 frames,
inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dense-field Mpixel/s @512² & 4K: plain FP32 vs BF16+learned P2S at fixed err"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
N_TRAIN = 2_000_000
N_HELDOUT = 100_000
TRAIN_BATCH = 8192

H = W = 512
C = 3
G = 1024
FRAMES = 16
K = 100
T = 33
P = 64
PITCH = 0.125
DR_CYCLE = (1.0, 2.0, 4.0)
N_BASIS_PSF = 20000


def kernel_work(name, frames):
    """Algorithmic work of one launch-set of `name` for `frames` frames:
    (bound, amount, unit).  Bytes are compulsory HBM traffic; flops count the
    arithmetic of the algorithm as specified (not instructions issued)."""
    px = frames * H * W
    if name == "k_sampler_cols":
        # write the row-cropped column-IFFT intermediate, 18 complex fields
        return "hbm", frames * 18 * H * G * 8, "B"
    if name == "k_sampler_rows_mix":
        # read the intermediate, write 35 coefficient planes
        return "hbm", frames * (18 * H * G * 8 + 35 * H * W * 4), "B"
    if name == "k_psf64":
        n_ap = 797  # pupil samples strictly inside the aperture (P = 64)
        phase = 2 * 33 * n_ap
        fft32 = 80 * 10 + 32 * 6          # radix-2 butterflies + pre-twiddle
        dft = 31 * 2 * fft32 + 33 * 2 * fft32 + 2 * 32 * 8
        return "alu", px * (phase + dft + 3 * T * T), "flop"
    if name == "k_project":
        return "alu", px * 2 * T * T * K, "flop"
    if name == "k_render_fp32":
        return "alu", px * (2 * K * T * T + 2 * C * T * T), "flop"
    if name == "k_warp":
        return "hbm", px * (8 + 4 * C + 4 * C), "B"
    if name == "k_mlp_infer":
        return "mfma", px * 2 * (35 * 256 + 2 * 256 * 256 + 256 * K), "flop"
    if name == "k_render_bf16":
        return "mfma", px * (2 * K * T * T + 2 * C * T * T), "flop"
    return None


def summarize(rep, steps, frames, traffic=True):
    """Per-kernel roofline entries from the tracer's {name: (launches, ms)}."""
    kernels = {}
    for name, (n, tot) in rep.items():
        w = kernel_work(name, frames)
        per_step = n / steps
        avg_ms = tot / n
        ent = {"launches_per_step": per_step, "avg_ms": round(avg_ms, 4),
               "ms_per_step": round(tot / steps, 4)}
        if w:
            bound, amount, unit = w
            per_launch = amount / per_step
            if bound == "hbm":
                ach = per_launch / (avg_ms * 1e-3) / 1e9
                ent.update(bound="hbm", achieved=round(ach, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                           frac=round(ach / PEAK_HBM_GBS, 4))
            else:
                peak = PEAK_BF16_TFLOPS if bound == "mfma" else PEAK_FP32_TFLOPS
                ach = per_launch / (avg_ms * 1e-3) / 1e12
                ent.update(bound=bound, achieved=round(ach, 3), peak=peak, unit="TFLOP/s",
                           frac=round(ach / peak, 4))
        kernels[name] = ent
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    d = kernels[dom]
    roof = {"kernel": dom, "bound": d.get("bound"), "achieved": d.get("achieved"),
            "peak": d.get("peak"), "unit": d.get("unit"), "frac": d.get("frac"),
            "traffic": measured_traffic(dom, d["launches_per_step"]) if traffic else None}
    return kernels, roof


def source_hash(kernel):
    files = {"k_sampler_cols": "sampler.hip", "k_sampler_rows_mix": "sampler.hip",
             "k_psf64": "psf.hip", "k_project": "psf.hip", "k_render_fp32": "render.hip",
             "k_warp": "render.hip"}
    f = files.get(kernel)
    if f is None:
        return None
    path = os.path.join(ROOT, "paper_2210_06713_amd", "csrc", f)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel, launches_per_step):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path)).get(kernel)
    except Exception:
        return None
    if not d or d.get("src_hash") != source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline():
    """The FP64 oracle on a bounded sample of the same workload, BLAS pinned
    to one thread: the sampler for one full 512 x 512 frame (grid 1024, plan
    tables excluded) plus exact P2S, basis blur and warp on a 64 x 64 block of
    that frame, extrapolated by pixel count to the full frame.  The oracle
    uses its own K = 100 PCA basis (built untimed from 400 oracle PSFs); the
    timing does not depend on the basis values."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import psf as opsf, render as orender, sampler as osamp, spectra as ospec
    from oracle import zernike as ozern
    import synthetic
    A, _ = opsf.basis_draws(400, seed=1)
    basis_np, _ = opsf.pca_basis(opsf.psf_batch(A, P, T), K)
    with threadpool_limits(limits=1):
        S = ospec.all_spectra(G, G, PITCH, 2)          # plan-time, not timed
        L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
        t0 = time.perf_counter()
        y = osamp.unit_fields(S, H, W, 0, 0)
        z = osamp.mix(y, L, 2.0)
        t_samp = time.perf_counter() - t0
        b = 64
        img = synthetic.test_image(C, b, b, 16, 0).astype(np.float64)
        zc = z[:, :b, :b]
        t0 = time.perf_counter()
        beta = opsf.psf_field(zc, P, T, basis_np)
        out = orender.render_frame(img, zc, beta, basis_np, T)
        t_block = time.perf_counter() - t0
    t_frame = t_samp + t_block * (H * W) / (b * b)
    return {"value": round(H * W / t_frame / 1e6, 6), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"FP64 oracle, 1 thread: sampler on one full {H}x{W} frame (G={G}) "
                       f"{t_samp:.2f} s + exact P2S/blur/warp on a 64x64x{C} block "
                       f"{t_block:.2f} s, extrapolated to the frame ({t_frame:.1f} s/frame)")}


BATCH_SIZES = ((24, 256, 256, 512, 512), (24, 512, 512, 1024, 1024), (16, 768, 1024, 2048, 2048))


def batched_graph(tsim, basis, net, steps):
    """Mixed-size batch (24 x 256^2, 24 x 512^2, 16 x 768x1024, 3 channels,
    per-frame D/r0 ~ U[1, 4]) in the learned BF16 form, captured once into a
    HIP graph and replayed: whole-batch Mpixel/s."""
    import numpy as np
    import torch
    import synthetic
    dev = torch.device("cuda:0")
    kp = 32 if K <= 32 else 64 if K <= 64 else 112 if K <= 112 else 128
    work = []
    for i, (F, Hb, Wb, Gh, Gw) in enumerate(BATCH_SIZES):
        pl = tsim.Plan(Hb, Wb, C, Gh, Gw, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis,
                       p2s_mode=tsim.P2S_LEARNED, precision=tsim.BF16)
        tsim.plan_set_mlp(pl, net)
        img = torch.tensor(np.repeat(synthetic.test_image(C, Hb, Wb, 16, i)[None], F, 0), device=dev)
        work.append(dict(pl=pl, F=F, img=img, dr=list(synthetic.d_over_r0_uniform(F, 1.0, 4.0, i)),
                         zern=torch.empty((F, 35, Hb, Wb), device=dev),
                         beta=torch.empty((F, Hb, Wb, kp), dtype=torch.bfloat16, device=dev),
                         blur=torch.empty((F, C, Hb, Wb), device=dev),
                         out=torch.empty((F, C, Hb, Wb), device=dev), ws=pl.workspace(F)))

    def run_all():
        for w in work:
            w["pl"].sample_zernike(w["dr"], 3, 0, w["zern"], w["ws"])
            w["pl"].p2s(w["zern"], w["beta"], w["ws"])
            w["pl"].render(w["img"], w["beta"], w["blur"])
            w["pl"].warp(w["blur"], w["zern"], w["out"])

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run_all()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run_all()
    g.replay()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        g.replay()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    px = sum(F * Hb * Wb for (F, Hb, Wb, _, _) in BATCH_SIZES)
    return {"workload": "64 frames: 24x256^2 (G=512), 24x512^2 (G=1024), 16x768x1024 (G=2048), "
                        "3 channels, D/r0 ~ U[1,4], learned BF16 form, one HIP graph",
            "value": round(px / (ms * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_batch": round(ms, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-steps", type=int, default=12000)
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); frames shard "
              "independently across GPUs, so the per-GPU figure is the one reported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2210_06713_amd as tsim
    import synthetic

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_setup = time.perf_counter()
    probe = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis_k=K)
    basis, eig = probe.basis_build(N_BASIS_PSF, seed=0, dr_lo=0.5, dr_hi=5.0)
    probe.close()
    plan = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis)
    setup_s = time.perf_counter() - t_setup

    img = torch.tensor(np.repeat(synthetic.test_image(C, H, W, 16, 0)[None], FRAMES, 0), device=dev)
    zern = torch.empty((FRAMES, 35, H, W), dtype=torch.float32, device=dev)
    drs = [DR_CYCLE[i % 3] for i in range(FRAMES)]

    def run(pl, beta, steps, warmup):
        """Time `steps` whole-path steps after `warmup`; returns (ms/step,
        tracer report, output of the last step)."""
        blur = torch.empty((FRAMES, C, H, W), dtype=torch.float32, device=dev)
        out = torch.empty_like(blur)
        ws = pl.workspace(FRAMES)

        def step(i):
            pl.sample_zernike(drs, 0, i * FRAMES, zern, ws)
            pl.p2s(zern, beta, ws)
            pl.render(img, beta, blur)
            pl.warp(blur, zern, out)

        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        tsim.trace_enable(True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for i in range(steps):
            step(warmup + i)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        rep = tsim.trace_report()
        tsim.trace_enable(False)
        if not torch.isfinite(out).all():
            raise RuntimeError("non-finite output")
        # the last step rendered frames (warmup + steps - 1) * FRAMES ...; rerun step 0 for a
        # fixed comparison frame set
        step(0)
        torch.cuda.synchronize()
        return ms, rep, out.clone()

    # ---- plain FP32 form (exact P2S) ----
    beta32 = torch.empty((FRAMES, H, W, K), dtype=torch.float32, device=dev)
    ms, rep, out_plain = run(plan, beta32, args.steps, args.warmup)
    kernels, roofline = summarize(rep, args.steps, FRAMES)
    value = FRAMES * H * W / (ms * 1e-3) / 1e6

    # ---- BF16 + learned form ----
    learned = None
    if not args.no_learned:
        t0 = time.perf_counter()
        plan_l = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis,
                           p2s_mode=tsim.P2S_LEARNED, precision=tsim.BF16)
        z_tr, b_tr = tsim.make_training_data(plan_l, N_TRAIN, seed=1)
        net = tsim.Mlp(plan_l, batch=TRAIN_BATCH, seed=0)
        net.fit_output(b_tr)
        t1 = time.perf_counter()
        losses = net.train(z_tr, b_tr, args.train_steps, lr_max=1e-3, lr_min=1e-5)
        train_s = time.perf_counter() - t1
        tsim.plan_set_mlp(plan_l, net)
        del z_tr, b_tr
        z_te, b_te = tsim.make_training_data(plan_l, N_HELDOUT, seed=2)
        pred = tsim.mlp_predict(plan_l, z_te)
        torch.cuda.synchronize()
        err = (torch.linalg.vector_norm(pred - b_te, dim=1)
               / torch.linalg.vector_norm(b_te, dim=1)).cpu().numpy()
        setup_l = time.perf_counter() - t0
        kp = 32 if K <= 32 else 64 if K <= 64 else 112 if K <= 112 else 128
        beta16 = torch.empty((FRAMES, H, W, kp), dtype=torch.bfloat16, device=dev)
        ms_l, rep_l, out_l = run(plan_l, beta16, args.steps, args.warmup)
        kern_l, roof_l = summarize(rep_l, args.steps, FRAMES, traffic=False)
        mse = float(torch.mean((out_l - out_plain) ** 2))
        learned = {"value": round(FRAMES * H * W / (ms_l * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
                   "ms_per_step": round(ms_l, 3), "dtype": "bf16 MFMA, fp32 accumulate",
                   "speedup_vs_plain_fp32": round(ms / ms_l, 2),
                   "psf_rel_err_mean": round(float(err.mean()), 5),
                   "psf_rel_err_median": round(float(np.median(err)), 5),
                   "psf_rel_err_p95": round(float(np.percentile(err, 95)), 5),
                   "psf_err_definition": "||beta_net - beta_exact|| / ||beta_exact|| on 1e5 held-out "
                                         "pairs (= relative L2 error of the projected PSF)",
                   "image_psnr_db_vs_plain_fp32": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None,
                   "train": {"pairs": N_TRAIN, "batch": TRAIN_BATCH, "steps": args.train_steps,
                             "seconds": round(train_s, 2),
                             "loss_first": float(losses[:10].mean()),
                             "loss_last": float(losses[-10:].mean())},
                   "setup_s": round(setup_l, 2), "roofline": roof_l, "kernels": kern_l}

        if not args.no_batched:
            learned["batched_graph"] = batched_graph(tsim, basis, net, args.steps)

    line = {"metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "512x512x3 float32, 16 frames, D/r0 cycling 1/2/4, Noll 2..36 "
                                   "on a 1024x1024 grid, exact 64x64-pupil PSFs, K=100 33x33 PCA "
                                   "basis, FP32 basis blur + bilinear tilt warp (plain FP32 form)",
                       "frames_per_step": FRAMES, "H": H, "W": W, "C": C, "grid": G, "K": K,
                       "T": T, "pupil": P},
            "roofline": roofline, "kernels": kernels, "learned_bf16": learned,
            "setup_s": round(setup_s, 2)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

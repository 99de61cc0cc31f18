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
import multiprocessing
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
TRAIN_LR = 2e-3

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

# the two single-frame-size workloads; `chunk` frames go through each call
# "counters": the name the workload's rocprofv3 byte counts are filed under in
# profiles/traffic.json (per launch, taken at the same launch shapes)
S512 = dict(H=H, W=W, C=C, G=G, T=T, P=P, K=K, frames=FRAMES, chunk=FRAMES, drs=DR_CYCLE,
            square=16, counters="512x512x3_16frames")
S4K = dict(H=2160, W=3840, C=3, G=4096, T=65, P=128, K=100, frames=30, chunk=6, drs=(3.0,),
           square=64, counters="3840x2160x3_6frames")


def n_aperture(P):
    """Pupil samples strictly inside the aperture (diameter P/2 samples)."""
    r = P // 4
    return sum(1 for y in range(-r, r) for x in range(-r, r) if x * x + y * y < r * r)


def kernel_work(name, frames, s):
    """Algorithmic work of one launch-set of `name` for `frames` frames of
    shape `s`: (bound, amount, unit).  Bytes are compulsory HBM traffic;
    flops count the arithmetic of the algorithm as specified (not
    instructions issued)."""
    h, w, c, g, t, k = s["H"], s["W"], s["C"], s["G"], s["T"], s["K"]
    px = frames * h * w
    if name == "k_sampler_cols":
        # write the row-cropped column-IFFT intermediate, 18 complex fields
        return "hbm", frames * 18 * h * g * 8, "B"
    if name == "k_sampler_rows_mix":
        # read the intermediate, write 35 coefficient planes
        return "hbm", frames * (18 * h * g * 8 + 35 * h * w * 4), "B"
    if name in ("k_psf64", "k_psf128"):
        n = 32 if name == "k_psf64" else 64      # register FFT length
        rows = n - 1                              # window rows inside the aperture
        fft = (n // 2) * int(math.log2(n)) * 10 + n * 6   # butterflies + pre-twiddle
        phase = 2 * 33 * n_aperture(2 * n)
        dft = rows * 2 * fft + n * 2 * fft + (n + 1) * n * 8   # + the direct edge column
        return "alu", px * (phase + dft + 3 * t * t), "flop"
    if name == "k_project":
        # read each pixel's T x T PSF, write its K weights (the contraction
        # runs on the 16-bit matrix cores, as three FP16 products per term)
        return "hbm", px * (t * t * 4 + k * 4), "B"
    if name == "k_render_fp32":
        # the plain blur's products run on the 16-bit matrix cores, three
        # FP16 products per FP32 term: executed flops against the FP16 peak
        return "mfma", px * 3 * 2 * k * t * t, "flop"
    if name == "k_warp":
        return "hbm", px * (8 + 4 * c + 4 * c), "B"
    if name == "k_subharmonic_add":
        # read and write the 8 coefficient planes of the two tilt groups
        return "hbm", px * 8 * 4 * 2, "B"
    if name == "k_ar_scan":
        # read each fresh frame and write the correlated one, 35 planes
        return "hbm", px * 2 * 35 * 4, "B"
    if name == "k_otf64":
        # per pixel: the phase at the aperture samples (35 modes), the full
        # 64 x 64 DFT of the pupil (31 window rows and 64 columns, each two
        # pruned 32-point DFTs) and |.|^2
        fft = 16 * 5 * 10 + 32 * 6
        return "alu", px * (2 * 35 * n_aperture(64) + 31 * 2 * fft + 64 * 2 * fft + 3 * 64 * 64), "flop"
    if name == "k_mlp_infer":
        return "mfma", px * 2 * (35 * 256 + 2 * 256 * 256 + 256 * k), "flop"
    if name == "k_render_bf16":
        return "mfma", px * (2 * k * t * t + 2 * c * t * t), "flop"
    return None


def summarize(rep, steps, frames, s, traffic=False):
    """Per-kernel roofline entries from the tracer's {name: (launches, ms)}."""
    kernels = {}
    for name, (n, tot) in rep.items():
        w = kernel_work(name, frames, s)
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
            "traffic": measured_traffic(dom, s["counters"]) if traffic else None}
    return kernels, roof


def source_hash(kernel):
    files = {"k_sampler_cols": "sampler.hip", "k_sampler_rows_mix": "sampler.hip",
             "k_psf64": "psf.hip", "k_psf128": "psf.hip", "k_project": "project.hip",
             "k_render_fp32": "render_bf16.hip", "k_render_bf16": "render_bf16.hip",
             "k_mlp_infer": "mlp.hip", "k_warp": "render.hip"}
    f = files.get(kernel)
    if f is None:
        return None
    csrc = os.path.join(ROOT, "paper_2210_06713_amd", "csrc")
    # the kernel's file and the shared device header it includes
    return hashlib.sha256(open(os.path.join(csrc, f), "rb").read() +
                          open(os.path.join(csrc, "common.cuh"), "rb").read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    the workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path)).get(workload, {}).get("kernels", {}).get(kernel)
    except Exception:
        return None
    if not d or d.get("src_hash") != source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


# ---- CPU baseline: the FP64 oracle, unchanged, run by a pool of worker
# processes (one BLAS thread each) over independent pieces of the workload.
_ORC = {}
_ORC_PARENT = {}     # the oracle's spectra and mixing matrix, kept for accuracy_vs_oracle


def _orc_init(basis_np, spectra_np, L_np):
    from threadpoolctl import threadpool_limits
    _ORC.update(basis=basis_np, S=spectra_np, L=L_np, lim=threadpool_limits(limits=1))


def _orc_sample(dr):
    from oracle import sampler as osamp
    y = osamp.unit_fields(_ORC["S"], H, W, 0, 0)
    return osamp.mix(y, _ORC["L"], dr)


def _orc_p2s(zband):
    from oracle import psf as opsf
    return opsf.psf_field(zband, P, T, _ORC["basis"])


def _orc_render(args):
    import numpy as np
    from oracle import render as orender
    import synthetic
    zern, beta, c = args
    img = synthetic.test_image(C, H, W, 16, 0)[c:c + 1].astype(np.float64)
    return orender.render_frame(img, zern, beta, _ORC["basis"], T)


def cpu_baseline(frames_sample=3):
    """The FP64 oracle on the 512 x 512 x 3 workload, one full frame per
    D/r0 in (1, 2, 4) (sampler, exact P2S of all 262 144 pixels, basis blur
    and warp), spread over a pool of worker processes: the three frames'
    samplers, then the P2S in 32-row bands, then the blur and warp per
    channel.  The oracle's K = 100 basis and the sampler's spectra are plan
    work, built before the clock starts."""
    import concurrent.futures as cf
    import numpy as np
    from oracle import psf as opsf, spectra as ospec, zernike as ozern
    workers = max(1, min(16, os.cpu_count() or 1))
    A, _ = opsf.basis_draws(400, seed=1)
    basis_np, _ = opsf.pca_basis(opsf.psf_batch(A, P, T), K)
    S = ospec.all_spectra(G, G, PITCH, 2)
    L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    drs = list(DR_CYCLE)[:frames_sample]
    band = 32
    # forked before anything touches the GPU (main() runs this first)
    ctx = multiprocessing.get_context("fork")
    with cf.ProcessPoolExecutor(workers, mp_context=ctx, initializer=_orc_init,
                                initargs=(basis_np, S, L)) as ex:
        list(ex.map(_orc_p2s, [np.zeros((35, 1, 8))] * workers))      # start the workers
        t0 = time.perf_counter()
        zs = list(ex.map(_orc_sample, drs))
        t1 = time.perf_counter()
        bands = [z[:, y:y + band] for z in zs for y in range(0, H, band)]
        betas = list(ex.map(_orc_p2s, bands))
        t2 = time.perf_counter()
        per = H // band
        full = [np.concatenate(betas[i * per:(i + 1) * per], axis=0) for i in range(len(zs))]
        outs = list(ex.map(_orc_render, [(zs[i], full[i], c) for i in range(len(zs)) for c in range(C)]))
        t3 = time.perf_counter()
    assert all(np.isfinite(o).all() for o in outs)
    _ORC_PARENT.update(S=S, L=L)
    wall = t3 - t0
    px = len(drs) * H * W
    return {"value": round(px / wall / 1e6, 6), "unit": "Mpixel/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"FP64 oracle in {workers} worker processes (1 thread each): {len(drs)} full "
                       f"{H}x{W}x{C} frames, D/r0 {drs}, G={G}: sampler {t1 - t0:.1f} s, exact "
                       f"P2S {t2 - t1:.1f} s, blur + warp {t3 - t2:.1f} s wall "
                       f"({wall / len(drs):.1f} s/frame)")}


BATCH_SIZES = ((24, 256, 256, 512, 512), (24, 512, 512, 1024, 1024), (16, 768, 1024, 2048, 2048))


ACC_BLOCK = (240, 272, 240, 272)    # rows y0..y1, columns x0..x1 of the compared block


def accuracy_vs_oracle(basis, zern_gpu, outs_gpu):
    """Part of the CPU-baseline leg: the FP64 oracle's fields and output
    pixels for the first three frames of the timed 512^2 workload (frame
    counters 0, 1, 2; D/r0 1, 2, 4; seed 0), with the GPU plan's own basis
    as data, against the GPU's.  Fields: relative L2 error over each whole
    frame.  Images: PSNR (peak 1) and relative L2 error over a 32 x 32 block
    of all three channels, for each form in `outs_gpu` ({form: [3][C][H][W]}).
    The block's blur needs the weights only at the bilinear taps of its
    pixels, so the oracle computes exact PSFs there alone."""
    import numpy as np
    from oracle import psf as opsf, render as orender, sampler as osamp, spectra as ospec, zernike as ozern
    import synthetic
    S = _ORC_PARENT.get("S")
    if S is None:
        S = ospec.all_spectra(G, G, PITCH, 2)
    L = _ORC_PARENT.get("L")
    if L is None:
        L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    y0, y1, x0, x1 = ACC_BLOCK
    ys, xs = [a.ravel() for a in np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")]
    img = synthetic.test_image(C, H, W, 16, 0).astype(np.float64)
    res = {"block": f"rows {y0}..{y1 - 1}, columns {x0}..{x1 - 1}, 3 channels",
           "frames": "frame counters 0, 1, 2 (D/r0 1, 2, 4), seed 0"}
    field_err, ref_px = [], []
    for f, dr in enumerate(DR_CYCLE):
        z = osamp.mix(osamp.unit_fields(S, H, W, f, 0), L, dr)
        zg = zern_gpu[f].astype(np.float64)
        field_err.append(float(np.linalg.norm(zg - z) / np.linalg.norm(z)))
        tx, ty = orender.tilt_shift(z)
        taps = set()
        for y, x in zip(ys, xs):
            py, px = y - ty[y, x], x - tx[y, x]
            fy, fx = int(np.floor(py)), int(np.floor(px))
            for yy in (fy, fy + 1):
                for xx in (fx, fx + 1):
                    taps.add((min(max(yy, 0), H - 1), min(max(xx, 0), W - 1)))
        ty_, tx_ = np.array(sorted(taps)).T
        beta = opsf.project(opsf.psf_batch(z[:, ty_, tx_].T, P, T), basis)
        out = np.empty((C, len(ys)))
        for c in range(C):
            blur = np.zeros((H, W))
            blur[ty_, tx_] = orender.render_at(img[c], beta, basis, T, ty_, tx_)
            out[c] = orender.warp_at(blur, tx[ys, xs], ty[ys, xs], ys, xs)
        ref_px.append(out)
    res["field_rel_err_per_frame"] = [float(f"{e:.3g}") for e in field_err]
    for form, outs in outs_gpu.items():
        per = []
        for f in range(len(DR_CYCLE)):
            got = outs[f][:, ys, xs].astype(np.float64)
            ref = ref_px[f]
            mse = float(((got - ref) ** 2).mean())
            per.append({"d_over_r0": DR_CYCLE[f],
                        "psnr_db": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None,
                        "rel_err": float(f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.3g}")})
        res[form] = per
    return res


def batched_graph(tsim, basis, net, steps):
    """Mixed-size batch (24 x 256^2, 24 x 512^2, 16 x 768x1024, 3 channels,
    per-frame D/r0 ~ U[1, 4]) in the learned BF16 form through the library's
    batch API (tsim_batch_create records every call into one HIP graph,
    tsim_batch_launch replays it): whole-batch Mpixel/s."""
    import numpy as np
    import torch
    import synthetic
    dev = torch.device("cuda:0")
    kp = 32 if K <= 32 else 64 if K <= 64 else 112 if K <= 112 else 128
    items, plans = [], []
    f0 = 0
    for i, (F, Hb, Wb, Gh, Gw) in enumerate(BATCH_SIZES):
        pl = tsim.Plan(Hb, Wb, C, Gh, Gw, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis,
                       p2s_mode=tsim.P2S_LEARNED, precision=tsim.BF16)
        tsim.plan_set_mlp(pl, net)
        plans.append(pl)
        img = torch.tensor(np.repeat(synthetic.test_image(C, Hb, Wb, 16, i)[None], F, 0), device=dev)
        items.append(dict(plan=pl, d_over_r0=list(synthetic.d_over_r0_uniform(F, 1.0, 4.0, i)), frame0=f0,
                          img=img, zern=torch.empty((F, 35, Hb, Wb), device=dev),
                          beta=torch.empty((F, Hb, Wb, kp), dtype=torch.bfloat16, device=dev),
                          blur=torch.empty((F, C, Hb, Wb), device=dev),
                          out=torch.empty((F, C, Hb, Wb), device=dev), ws=pl.workspace(F)))
        f0 += F
    batch = tsim.Batch(items, 3)
    batch.launch()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        batch.launch()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    batch.close()
    for pl in plans:
        pl.close()
    px = sum(F * Hb * Wb for (F, Hb, Wb, _, _) in BATCH_SIZES)
    return {"workload": "64 frames: 24x256^2 (G=512), 24x512^2 (G=1024), 16x768x1024 (G=2048), "
                        "3 channels, D/r0 ~ U[1,4], learned BF16 form, one library-built HIP graph "
                        "(tsim_batch_create / tsim_batch_launch)",
            "value": round(px / (ms * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_batch": round(ms, 3)}


def time_then_trace(tsim, torch, fn, steps, host_clock=False):
    """ms per call of fn(i), i = 0..steps-1, timed with tracing off (HIP
    events on the current stream, or the host clock for calls that
    synchronise), then the library's per-kernel report (launch counts and
    event-timed durations on each launch's stream) over `steps` further
    calls fn(steps + i) with tracing on."""
    torch.cuda.synchronize()
    if host_clock:
        t0 = time.perf_counter()
        for i in range(steps):
            fn(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    else:
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(steps):
            fn(i)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
    tsim.trace_enable(True)
    for i in range(steps):
        fn(steps + i)
    torch.cuda.synchronize()
    rep = tsim.trace_report()
    tsim.trace_enable(False)
    return ms, rep


class Workload:
    """Frames of one shape: a repeated synthetic scene, per-frame D/r0, and
    `chunk`-frame buffers that each call works on."""

    def __init__(self, torch, synthetic, s, dev):
        import numpy as np
        self.torch, self.s, self.dev = torch, s, dev
        n = s["chunk"]
        self.img = torch.tensor(np.repeat(synthetic.test_image(s["C"], s["H"], s["W"], s["square"], 0)[None],
                                          n, 0), device=dev)
        self.zern = torch.empty((n, 35, s["H"], s["W"]), dtype=torch.float32, device=dev)
        self.blur = torch.empty((n, s["C"], s["H"], s["W"]), dtype=torch.float32, device=dev)
        self.out = torch.empty_like(self.blur)

    def run(self, tsim, pl, beta, steps, warmup, frames):
        """Time `steps` whole-path steps of `frames` frames after `warmup`;
        returns (ms/step, tracer report, output of the first chunk of step 0)."""
        torch, s = self.torch, self.s
        n = s["chunk"]
        ws = pl.workspace(n)
        drs = s["drs"]
        # the sampler's launch forms, chosen by the library's autotuner on
        # these buffers (the fields do not depend on the choice)
        self.tuning = pl.autotune(n, self.zern[:n], ws)

        def chunk(i, c0):
            m = min(n, frames - c0)
            f0 = i * frames + c0
            z, b, bl, o = self.zern[:m], beta[:m], self.blur[:m], self.out[:m]
            pl.sample_zernike([drs[(c0 + f) % len(drs)] for f in range(m)], 0, f0, z, ws)
            pl.p2s(z, b, ws)
            pl.render(self.img[:m], b, bl)
            pl.warp(bl, z, o)

        def step(i):
            for c0 in range(0, frames, n):
                chunk(i, c0)

        for i in range(warmup):
            step(i)
        ms, rep = time_then_trace(tsim, torch, lambda i: step(warmup + i), steps)
        if not torch.isfinite(self.out).all():
            raise RuntimeError("non-finite output")
        chunk(0, 0)              # fixed frames (the first chunk of step 0) for comparing forms
        torch.cuda.synchronize()
        self.zern_first = self.zern[:min(3, n, frames)].cpu().numpy()
        return ms, rep, self.out[:min(n, frames)].clone()


def frame_call(tsim, torch, wl, pl, s, steps, frames, group=None):
    """The same frames through the one-call path (tsim_frame), at the plan's
    default group unless one is given: the whole step is one call, and the
    fields, weights and blurred frames of one group at a time live in its
    workspace."""
    g = pl.frame_group() if group is None else group
    ws = pl.frame_workspace(g)
    drs = s["drs"]
    img = wl.img[:1].expand(frames, -1, -1, -1).contiguous() if frames > wl.img.shape[0] else wl.img[:frames]
    out = torch.empty_like(img)
    d = [drs[f % len(drs)] for f in range(frames)]
    pl.frame(d, 0, 0, img, out, ws, group=g)
    ms, rep = time_then_trace(tsim, torch, lambda i: pl.frame(d, 0, (1 + i) * frames, img, out, ws, group=g),
                              steps)
    kern, _ = summarize(rep, steps, frames, s, traffic=False)
    px = s["H"] * s["W"]
    sep = frames * px * (35 * 4 + pl.KP * 2 + s["C"] * 4)
    res = {"value": round(frames * px / (ms * 1e-3) / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(ms, 3),
           "frames_per_call": frames, "group": g, "workspace_mib": round(pl.frame_workspace_bytes(g) / 2**20, 1),
           "fields_weights_blur_of_all_frames_mib": round(sep / 2**20, 1), "kernels": kern}
    del ws, img, out
    return res


def train_network(tsim, torch, np, plan_l, train_steps):
    """The learned form's network: 2M exact (Zernike, weight) pairs from the
    plan's own PSF path, MSE training on the GPU, held-out PSF error."""
    t0 = time.perf_counter()
    z_tr, b_tr = tsim.make_training_data(plan_l, N_TRAIN, seed=1)
    net = tsim.Mlp(plan_l, batch=TRAIN_BATCH, seed=0)
    net.fit_output(b_tr)
    t1 = time.perf_counter()
    losses = net.train(z_tr, b_tr, train_steps, lr_max=TRAIN_LR, lr_min=1e-5)
    train_s = time.perf_counter() - t1
    tsim.plan_set_mlp(plan_l, net)
    del z_tr, b_tr

    def psf_err(z_te, b_te):
        pred = tsim.mlp_predict(plan_l, z_te)
        torch.cuda.synchronize()
        return (torch.linalg.vector_norm(pred - b_te, dim=1)
                / torch.linalg.vector_norm(b_te, dim=1)).cpu().numpy()

    err = psf_err(*tsim.make_training_data(plan_l, N_HELDOUT, seed=2))
    # the timed workload's own turbulence strengths
    at = {str(d): round(float(psf_err(*tsim.make_training_data(plan_l, 20000, seed=3 + i, dr_lo=d,
                                                                dr_hi=d)).mean()), 5)
          for i, d in enumerate(DR_CYCLE)}
    info = {"psf_rel_err_mean": round(float(err.mean()), 5),
            "psf_rel_err_median": round(float(np.median(err)), 5),
            "psf_rel_err_p95": round(float(np.percentile(err, 95)), 5),
            "psf_rel_err_mean_at_d_over_r0": at,
            "psf_err_definition": "||beta_net - beta_exact|| / ||beta_exact|| on 1e5 held-out "
                                  "pairs, D/r0 ~ U[0.5, 5] (= relative L2 error of the projected PSF); "
                                  "and on 2e4 pairs at each D/r0 of the timed frames",
            "train": {"pairs": N_TRAIN, "batch": TRAIN_BATCH, "steps": train_steps, "lr_max": TRAIN_LR,
                      "seconds": round(train_s, 2),
                      "loss_first": float(losses[:10].mean()),
                      "loss_last": float(losses[-10:].mean())},
            "setup_s": round(time.perf_counter() - t0, 2)}
    return net, info


def kpad(k):
    return 32 if k <= 32 else 64 if k <= 64 else 112 if k <= 112 else 128


def psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None


def ar_sequence(tsim, torch, wl, s, steps):
    """Temporally correlated frames (auto-regression, alpha = 0.95) in
    6-frame chunks, each chunk continuing from the previous one's last frame:
    sampler + scan per chunk."""
    pl = tsim.Plan(s["H"], s["W"], s["C"], s["G"], s["G"], pixel_pitch_over_d=PITCH)
    n = s["chunk"]
    ws = pl.workspace(n)
    prev = torch.zeros_like(wl.zern[0])
    drs = [s["drs"][0]] * n

    def chunk(i):
        pl.sample_zernike_ar(drs, 0, i * n, 0.95, wl.zern, ws, zern_prev=prev, d_over_r0_prev=drs[0])
        prev.copy_(wl.zern[n - 1])

    chunk(0)
    ms, rep = time_then_trace(tsim, torch, lambda i: chunk(1 + i), steps)
    kern, roof = summarize(rep, steps, n, s, traffic=False)
    pl.close()
    return {"workload": f"{n} frames per chunk, alpha 0.95, continuing chunk to chunk",
            "value": round(n * s["H"] * s["W"] / (ms * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
            "ms_per_chunk": round(ms, 3), "kernels": kern}


STAT_LAG = 64


def subharmonic_sampler(tsim, torch, wl, s, steps):
    """The sampler alone on the 512^2 workload (16 frames per call), without
    and with three subharmonic levels for the tilt fields; then the spatial
    tilt statistics of the latter's frames (host-synchronous calls)."""
    n = s["chunk"]
    drs = [s["drs"][i % len(s["drs"])] for i in range(n)]
    out = {"workload": f"{n} frames of {s['H']}x{s['W']}, grid {s['G']}^2, sampler only"}
    for levels in (0, 3):
        pl = tsim.Plan(s["H"], s["W"], s["C"], s["G"], s["G"], pixel_pitch_over_d=PITCH,
                       subharmonic_levels=levels)
        ws = pl.workspace(n)
        pl.sample_zernike(drs, 0, 0, wl.zern, ws)
        ms, rep_ = time_then_trace(tsim, torch, lambda i: pl.sample_zernike(drs, 0, (1 + i) * n, wl.zern, ws),
                                   steps)
        kern, _ = summarize(rep_, steps, n, s, traffic=False)
        out[f"levels_{levels}"] = {"value": round(n * s["H"] * s["W"] / (ms * 1e-3) / 1e6, 3),
                                   "unit": "Mpixel/s", "ms_per_call": round(ms, 4), "kernels": kern}
        if levels:
            # spatial tilt statistics of these frames, lags 0..64 along x and y
            pl.tilt_stats(wl.zern, STAT_LAG)
            ms_s, rep_ = time_then_trace(tsim, torch, lambda i: pl.tilt_stats(wl.zern, STAT_LAG), steps,
                                         host_clock=True)
            kern_s, _ = summarize(rep_, steps, n, s, traffic=False)
            out["tilt_stats"] = {"max_lag": STAT_LAG, "frames": n,
                                 "value": round(n * s["H"] * s["W"] / (ms_s * 1e-3) / 1e6, 3),
                                 "unit": "Mpixel/s", "ms_per_call": round(ms_s, 4),
                                 "kernels": kern_s}
            # phase structure function over the aperture (device moments,
            # host quadratic form)
            pl.structure_function(wl.zern)
            ms_f, rep_ = time_then_trace(tsim, torch, lambda i: pl.structure_function(wl.zern), steps,
                                         host_clock=True)
            kern_f, _ = summarize(rep_, steps, n, s, traffic=False)
            out["structure_function"] = {"frames": n, "ms_per_call": round(ms_f, 4),
                                         "value": round(n * s["H"] * s["W"] / (ms_f * 1e-3) / 1e6, 3),
                                         "unit": "Mpixel/s", "kernels": kern_f}
            # long- and short-exposure OTFs (each pixel's full 64 x 64 pupil
            # spectrum on the device, inverse DFT of the mean on the host)
            for name, short in (("otf_long_exposure", False), ("otf_short_exposure", True)):
                pl.otf(wl.zern, short_exposure=short)
                ms_o, rep_ = time_then_trace(tsim, torch, lambda i: pl.otf(wl.zern, short_exposure=short),
                                             steps, host_clock=True)
                kern_o, _ = summarize(rep_, steps, n, s, traffic=False)
                out[name] = {"frames": n, "ms_per_call": round(ms_o, 4),
                             "value": round(n * s["H"] * s["W"] / (ms_o * 1e-3) / 1e6, 3),
                             "unit": "Mpixel/s", "kernels": kern_o}
        del ws
        pl.close()
    return out


def large_frame(tsim, torch, np, synthetic, dev, args):
    """3840 x 2160 x 3 frames, D/r0 = 3, 4096^2 grid, 128 x 128 pupil, K = 100
    basis of 65 x 65 kernels: a 30-frame sequence of independent draws per
    step in the learned BF16 form; the plain FP32 form on 6 frames per step
    (its exact PSFs cost about a second per frame)."""
    s = S4K
    t0 = time.perf_counter()
    probe = tsim.Plan(s["H"], s["W"], s["C"], s["G"], s["G"], pixel_pitch_over_d=PITCH, psf_t=s["T"],
                      pupil_n=s["P"], basis_k=s["K"])
    basis, _ = probe.basis_build(N_BASIS_PSF, seed=0, dr_lo=0.5, dr_hi=5.0)
    probe.close()
    basis_s = time.perf_counter() - t0
    wl = Workload(torch, synthetic, s, dev)
    n = s["chunk"]
    plan = tsim.Plan(s["H"], s["W"], s["C"], s["G"], s["G"], pixel_pitch_over_d=PITCH, psf_t=s["T"],
                     pupil_n=s["P"], basis=basis)
    beta32 = torch.empty((n, s["H"], s["W"], s["K"]), dtype=torch.float32, device=dev)
    f_plain = n
    st_plain = max(1, min(args.steps, 2))
    ms_p, rep_p, out_p = wl.run(tsim, plan, beta32, st_plain, 1, f_plain)
    kern_p, roof_p = summarize(rep_p, st_plain, f_plain, s, traffic=True)
    del beta32
    plan.close()
    px = s["H"] * s["W"]
    plain = {"value": round(f_plain * px / (ms_p * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
             "ms_per_step": round(ms_p, 3), "frames_per_step": f_plain, "steps": st_plain,
             "warmup": 1, "dtype": "f32", "roofline": roof_p, "kernels": kern_p}
    out = {"workload": "3840x2160x3 float32, D/r0 = 3, Noll 2..36 on a 4096x4096 grid, "
                       "128x128-pupil PSFs, K=100 65x65 PCA basis, blur + bilinear tilt warp",
           "basis_build_s": round(basis_s, 2), "plain_fp32": plain}
    if not args.no_learned:
        plan_l = tsim.Plan(s["H"], s["W"], s["C"], s["G"], s["G"], pixel_pitch_over_d=PITCH,
                           psf_t=s["T"], pupil_n=s["P"], basis=basis, p2s_mode=tsim.P2S_LEARNED,
                           precision=tsim.BF16)
        net, info = train_network(tsim, torch, np, plan_l, args.train_steps)
        beta16 = torch.empty((n, s["H"], s["W"], kpad(s["K"])), dtype=torch.bfloat16, device=dev)
        ms_l, rep_l, out_l = wl.run(tsim, plan_l, beta16, args.steps, args.warmup, s["frames"])
        kern_l, roof_l = summarize(rep_l, args.steps, s["frames"], s, traffic=True)
        learned = {"value": round(s["frames"] * px / (ms_l * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
                   "ms_per_step": round(ms_l, 3), "frames_per_step": s["frames"],
                   "steps": args.steps, "warmup": args.warmup,
                   "dtype": "bf16 MFMA, fp32 accumulate",
                   "speedup_vs_plain_fp32": round((ms_p / f_plain) / (ms_l / s["frames"]), 2),
                   "image_psnr_db_vs_plain_fp32": psnr(out_l, out_p)}
        learned.update(info)
        learned.update(roofline=roof_l, kernels=kern_l)
        del beta16
        if not args.no_frame_call:
            learned["frame_call"] = frame_call(tsim, torch, wl, plan_l, s, max(1, min(args.steps, 2)),
                                               s["frames"])
        out["learned_bf16"] = learned
        del net
        plan_l.close()
        out["ar_sequence"] = ar_sequence(tsim, torch, wl, s, args.steps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-steps", type=int, default=24000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-4k", action="store_true")
    ap.add_argument("--no-frame-call", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); frames shard "
              "independently across GPUs, so the per-GPU figure is the one reported",
              file=sys.stderr)
        sys.exit(2)

    # the oracle's CPU baseline first, in worker processes forked before this
    # process initialises the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    import numpy as np
    import torch
    import paper_2210_06713_amd as tsim
    import synthetic

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = S512
    t_setup = time.perf_counter()
    probe = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis_k=K)
    basis, eig = probe.basis_build(N_BASIS_PSF, seed=0, dr_lo=0.5, dr_hi=5.0)
    probe.close()
    plan = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis)
    setup_s = time.perf_counter() - t_setup
    wl = Workload(torch, synthetic, s, dev)

    # ---- plain FP32 form (exact P2S) ----
    beta32 = torch.empty((FRAMES, H, W, K), dtype=torch.float32, device=dev)
    ms, rep, out_plain = wl.run(tsim, plan, beta32, args.steps, args.warmup, FRAMES)
    wl_tuning = wl.tuning
    zern_first = wl.zern_first
    outs_first = {"plain_fp32": out_plain[:3].cpu().numpy()}
    kernels, roofline = summarize(rep, args.steps, FRAMES, s, traffic=True)
    value = FRAMES * H * W / (ms * 1e-3) / 1e6
    del beta32
    # the same step as one tsim_frame call, in groups of one P2S chunk
    frame_plain = None if args.no_frame_call else frame_call(tsim, torch, wl, plan, s, args.steps, FRAMES,
                                                              group=(1 << 20) // (H * W))

    # ---- BF16 + learned form ----
    learned = None
    if not args.no_learned:
        plan_l = tsim.Plan(H, W, C, G, G, pixel_pitch_over_d=PITCH, psf_t=T, pupil_n=P, basis=basis,
                           p2s_mode=tsim.P2S_LEARNED, precision=tsim.BF16)
        net, info = train_network(tsim, torch, np, plan_l, args.train_steps)
        beta16 = torch.empty((FRAMES, H, W, kpad(K)), dtype=torch.bfloat16, device=dev)
        ms_l, rep_l, out_l = wl.run(tsim, plan_l, beta16, args.steps, args.warmup, FRAMES)
        outs_first["learned_bf16"] = out_l[:3].cpu().numpy()
        kern_l, roof_l = summarize(rep_l, args.steps, FRAMES, s, traffic=True)
        learned = {"value": round(FRAMES * H * W / (ms_l * 1e-3) / 1e6, 3), "unit": "Mpixel/s",
                   "ms_per_step": round(ms_l, 3), "dtype": "bf16 MFMA, fp32 accumulate",
                   "speedup_vs_plain_fp32": round(ms / ms_l, 2),
                   "image_psnr_db_vs_plain_fp32": psnr(out_l, out_plain)}
        learned.update(info)
        learned.update(roofline=roof_l, kernels=kern_l)
        del beta16
        if not args.no_frame_call:
            learned["frame_call"] = frame_call(tsim, torch, wl, plan_l, s, args.steps, FRAMES)
        if not args.no_batched:
            learned["batched_graph"] = batched_graph(tsim, basis, net, args.steps)
        del net
        plan_l.close()
    plan.close()
    subh = subharmonic_sampler(tsim, torch, wl, s, args.steps)
    del wl
    torch.cuda.empty_cache()

    large = None
    if not args.no_4k:
        large = large_frame(tsim, torch, np, synthetic, dev, args)

    line = {"metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "512x512x3 float32, 16 frames, D/r0 cycling 1/2/4, Noll 2..36 "
                                   "on a 1024x1024 grid, exact 64x64-pupil PSFs, K=100 33x33 PCA "
                                   "basis, FP32 basis blur + bilinear tilt warp (plain FP32 form)",
                       "frames_per_step": FRAMES, "H": H, "W": W, "C": C, "grid": G, "K": K,
                       "T": T, "pupil": P},
            "sampler_forms": {"pass1_columns_per_block": wl_tuning[0], "pass2_form": wl_tuning[1]},
            "roofline": roofline, "kernels": kernels, "frame_call_plain_fp32": frame_plain,
            "learned_bf16": learned,
            "subharmonic_sampler": subh, "large_4k": large, "setup_s": round(setup_s, 2)}
    if cpu is not None:
        line["cpu_baseline"] = cpu
        line["accuracy_vs_fp64_oracle"] = accuracy_vs_oracle(basis, zern_first, outs_first)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Short, fixed workload for hardware-counter profiling of the hot path.

    rocprofv3 --pmc FETCH_SIZE -d OUT -o run -- python paper_2210_06713_amd/profile_driver.py
    rocprofv3 --pmc WRITE_SIZE -d OUT -o run -- python paper_2210_06713_amd/profile_driver.py
    python paper_2210_06713_amd/profile_driver.py --summarize OUT_FETCH OUT_WRITE profiles/
    python paper_2210_06713_amd/profile_driver.py --stats-md STATS.csv OUT.md "command" "title"

Runs ``--steps`` steps (default 2) of the 512 x 512 x 3, 16-frame workload
(or, with ``--workload 4k``, of 6-frame chunks of the 3840 x 2160 x 3
workload) in the plain FP32 form and in the learned BF16 form (network with
seeded random weights: the kernels' time and traffic do not depend on the
weight values), then one
element-wise copy of 256 MiB (read 256 MiB, write 256 MiB) whose counter
readings calibrate the per-kernel byte counts.  ``--summarize`` turns the two
counter runs into ``traffic.json`` (bytes per launch for each kernel, with
the hash of the kernel's source file and of the shared device header) and a
Markdown summary.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

CAL_BYTES = 256 << 20
# kernel symbol -> (name the launch tracer reports, source file)
SOURCES = {"k_sampler_cols": ("k_sampler_cols", "sampler.hip"),
           "k_sampler_rows_mix": ("k_sampler_rows_mix", "sampler.hip"),
           "k_psf64": ("k_psf64", "psf.hip"), "k_psf128": ("k_psf128", "psf.hip"),
           "k_project_mfma": ("k_project", "project.hip"),
           "k_render_f32m": ("k_render_fp32", "render_bf16.hip"),
           "k_render_bf16": ("k_render_bf16", "render_bf16.hip"),
           "k_mlp_infer": ("k_mlp_infer", "mlp.hip"), "k_warp": ("k_warp", "render.hip")}


WORKLOADS = {
    # H, W, C, grid, T, P, K, frames per call, D/r0 cycle, checker cell
    "512": (512, 512, 3, 1024, 33, 64, 100, 16, (1.0, 2.0, 4.0), 16),
    "4k": (2160, 3840, 3, 4096, 65, 128, 100, 6, (3.0,), 64),
}


def run(workload, steps):
    import numpy as np
    import torch
    import paper_2210_06713_amd as tsim
    import synthetic

    H, W, C, G, T, P, K, F, dr, sq = WORKLOADS[workload]
    dev = torch.device("cuda:0")
    probe = tsim.Plan(H, W, C, G, G, psf_t=T, pupil_n=P, basis_k=K)
    basis, _ = probe.basis_build(2000, seed=0)
    probe.close()
    img = torch.tensor(np.repeat(synthetic.test_image(C, H, W, sq, 0)[None], F, 0), device=dev)
    zern = torch.empty((F, 35, H, W), dtype=torch.float32, device=dev)
    blur = torch.empty((F, C, H, W), dtype=torch.float32, device=dev)
    out = torch.empty_like(blur)
    drs = [dr[i % len(dr)] for i in range(F)]
    for learned in (False, True):
        if learned:
            pl = tsim.Plan(H, W, C, G, G, psf_t=T, pupil_n=P, basis=basis, p2s_mode=tsim.P2S_LEARNED,
                           precision=tsim.BF16)
            net = tsim.Mlp(pl, batch=64, seed=0)
            tsim.plan_set_mlp(pl, net)
            beta = torch.empty((F, H, W, 112), dtype=torch.bfloat16, device=dev)
        else:
            pl = tsim.Plan(H, W, C, G, G, psf_t=T, pupil_n=P, basis=basis)
            beta = torch.empty((F, H, W, K), dtype=torch.float32, device=dev)
        ws = pl.workspace(F)
        for i in range(steps):
            pl.sample_zernike(drs, 0, i * F, zern, ws)
            pl.p2s(zern, beta, ws)
            pl.render(img, beta, blur)
            pl.warp(blur, zern, out)
            torch.cuda.synchronize()
            print(f"{workload} {'learned' if learned else 'plain'} step {i} done", flush=True)
        del beta, ws
        pl.close()
    src = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print("profile workload done", flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def _short(name):
    n = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0].split("<")[0].strip()


def _per_kernel(rows, counter):
    """{kernel: [KiB per dispatch]} for one counter (summed over dimensions)."""
    by_disp = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = (r.get("Dispatch_Id"), r.get("Kernel_Name"))
        by_disp[key] = by_disp.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (_, k), v in by_disp.items():
        out.setdefault(k, []).append(v)
    return out


def summarize(fetch_dir, write_dir, dst):
    fetch = _per_kernel(_rows(fetch_dir), "FETCH_SIZE")
    write = _per_kernel(_rows(write_dir), "WRITE_SIZE")

    def cal(d):
        for k, v in d.items():
            if "MulFunctor" in k:
                return (CAL_BYTES / 1024.0) / max(v)
        raise SystemExit("calibration copy not found")

    fr, wr = cal(fetch), cal(write)
    res = {"calibration": {"bytes": CAL_BYTES, "fetch_factor": round(fr, 4), "write_factor": round(wr, 4)}}
    lines = ["| kernel | dispatches | read MB/launch | write MB/launch | total MB/launch |",
             "|---|---:|---:|---:|---:|"]
    def median(v):
        v = sorted(v)
        return v[len(v) // 2]

    for k in sorted(set(fetch) | set(write)):
        s = _short(k)
        if s not in SOURCES:
            continue
        trace, src = SOURCES[s]
        f = fetch.get(k, [0.0])
        w = write.get(k, [0.0])
        # median over dispatches: the one-off basis-build launch is not typical
        rb = median(f) * 1024 * fr
        wb = median(w) * 1024 * wr
        csrc = os.path.join(ROOT, "paper_2210_06713_amd", "csrc")
        # the kernel's file and the shared device header it includes
        h = hashlib.sha256(open(os.path.join(csrc, src), "rb").read() +
                           open(os.path.join(csrc, "common.cuh"), "rb").read()).hexdigest()[:16]
        name = k.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].strip()
        res[trace] = {"kernel": name, "dispatches": len(f), "read_bytes_per_launch": round(rb),
                      "write_bytes_per_launch": round(wb), "bytes_per_launch": round(rb + wb),
                      "src_hash": h}
        lines.append(f"| {name} | {len(f)} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | {(rb + wb) / 1e6:.1f} |")
    os.makedirs(dst, exist_ok=True)
    json.dump(res, open(os.path.join(dst, "traffic.json"), "w"), indent=1)
    return res, lines, fr, wr


def stats_markdown(csv_path, dst, command, title):
    """rocprofv3 --stats kernel summary (kernel_stats.csv) -> Markdown table."""
    rows = list(csv.DictReader(open(csv_path)))
    out = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
           "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        n = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        if len(n) > 90:
            n = n[:87] + "..."
        out.append(f"| {n} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    with open(dst, "w") as f:
        f.write("\n".join(out) + "\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "DST"))
    ap.add_argument("--stats-md", nargs=4, metavar=("KERNEL_STATS_CSV", "DST_MD", "COMMAND", "TITLE"))
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="512")
    ap.add_argument("--steps", type=int, default=2)
    a = ap.parse_args()
    if a.stats_md:
        stats_markdown(*a.stats_md)
    elif a.summarize:
        res, lines, fr, wr = summarize(*a.summarize)
        print("\n".join(lines))
        print(f"calibration: fetch x{fr:.4f}, write x{wr:.4f}")
    else:
        run(a.workload, a.steps)

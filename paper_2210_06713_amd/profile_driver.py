"""Short, fixed workload for hardware-counter profiling of the hot path.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o run -- python paper_2210_06713_amd/profile_driver.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o run -- python paper_2210_06713_amd/profile_driver.py
    python paper_2210_06713_amd/profile_driver.py --summarize F W profiles/ [--workload 4k]
    rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS \
        SQ_ACTIVE_INST_VMEM GRBM_GUI_ACTIVE --output-format csv -d Q -o run -- python ...profile_driver.py
    python paper_2210_06713_amd/profile_driver.py --sq-summary Q OUT.md "command" "title"
    python paper_2210_06713_amd/profile_driver.py --stats-md STATS.csv OUT.md "command" "title"

Runs ``--steps`` steps (default 2) of the 512 x 512 x 3, 16-frame workload
(or, with ``--workload 4k``, of 6-frame chunks of the 3840 x 2160 x 3
workload) in the plain FP32 form and in the learned BF16 form (network with
seeded random weights: the kernels' time and traffic do not depend on the
weight values), then one element-wise copy of 256 MiB (read 256 MiB, write
256 MiB) whose counter readings calibrate the per-kernel byte counts.

``--summarize`` turns the two byte-counter runs into the workload's entry of
``traffic.json`` (bytes per launch for each kernel, with the hash of the
kernel's source file and of the shared device header) and a Markdown table.
``--sq-summary`` turns a run of shader-sequencer counters into per-kernel
busy fractions: matrix-core busy = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x 1024
SIMDs), and vector-ALU and LDS issue = SQ_ACTIVE_INST_* (in
quad cycles, per SIMD) x 4 / (cycles x 1024 SIMDs), with cycles = the
kernel's GRBM_GUI_ACTIVE, which rocprofv3 sums over the eight XCDs.
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
           "k_project_h3": ("k_project", "project.hip"),
           "k_render_h3": ("k_render_fp32", "render_bf16.hip"),
           "k_render_bf16": ("k_render_bf16", "render_bf16.hip"),
           "k_mlp_infer": ("k_mlp_infer", "mlp.hip"), "k_warp": ("k_warp", "render.hip")}


WORKLOADS = {
    # H, W, C, grid, T, P, K, frames per call, D/r0 cycle, checker cell
    "512": (512, 512, 3, 1024, 33, 64, 100, 16, (1.0, 2.0, 4.0), 16),
    "4k": (2160, 3840, 3, 4096, 65, 128, 100, 6, (3.0,), 64),
}
# the name each workload's counter figures are filed under
WORKLOAD_KEYS = {"512": "512x512x3_16frames", "4k": "3840x2160x3_6frames"}
N_SIMD = 1024      # 256 compute units x 4 SIMDs
N_XCD = 8


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


def summarize(fetch_dir, write_dir, dst, workload="512"):
    fetch = _per_kernel(_rows(fetch_dir), "FETCH_SIZE")
    write = _per_kernel(_rows(write_dir), "WRITE_SIZE")

    def cal(d):
        for k, v in d.items():
            if "MulFunctor" in k:
                return (CAL_BYTES / 1024.0) / max(v)
        raise SystemExit("calibration copy not found")

    fr, wr = cal(fetch), cal(write)
    entry = {"calibration": {"bytes": CAL_BYTES, "fetch_factor": round(fr, 4), "write_factor": round(wr, 4)},
             "kernels": {}}
    lines = ["| kernel | dispatches | read MB/launch | write MB/launch | total MB/launch |",
             "|---|---:|---:|---:|---:|"]

    for k in sorted(set(fetch) | set(write)):
        s = _short(k)
        if s not in SOURCES:
            continue
        trace, src = SOURCES[s]
        f = fetch.get(k, [0.0])
        w = write.get(k, [0.0])
        # median over dispatches: the one-off basis-build launch is not typical
        rb = _median(f) * 1024 * fr
        wb = _median(w) * 1024 * wr
        name = k.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].strip()
        entry["kernels"][trace] = {"kernel": name, "dispatches": len(f), "read_bytes_per_launch": round(rb),
                                   "write_bytes_per_launch": round(wb), "bytes_per_launch": round(rb + wb),
                                   "src_hash": source_hash(src)}
        lines.append(f"| {name} | {len(f)} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | {(rb + wb) / 1e6:.1f} |")
    os.makedirs(dst, exist_ok=True)
    path = os.path.join(dst, "traffic.json")
    res = {}
    if os.path.exists(path):
        res = json.load(open(path))
        if "calibration" in res:       # a single-workload file: start afresh
            res = {}
    key = WORKLOAD_KEYS[workload]
    res[key] = entry
    json.dump(res, open(path, "w"), indent=1, sort_keys=True)
    drv = "REPO/paper_2210_06713_amd/profile_driver.py"
    md = [f"# HBM traffic per launch: {key} (plain FP32 and learned BF16 forms)", "",
          "Commands (from the repository root, on one MI355X; one counter per run):", "", "```",
          f"cd /tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d FETCH -o run -- python -u {drv} "
          f"--workload {workload}",
          f"cd /tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d WRITE -o run -- python -u {drv} "
          f"--workload {workload}",
          f"python {drv} --summarize FETCH WRITE REPO/profiles/ --workload {workload}", "```", "",
          "The driver runs two steps of each form, then one element-wise copy of 256 MiB (read 256 MiB,",
          f"write 256 MiB) whose readings give the calibration: FETCH_SIZE x{fr:.4f}, WRITE_SIZE x{wr:.4f}",
          "(bytes = KiB reading x 1024 x factor). Each value is the median over the kernel's dispatches;",
          "traffic.json holds the same figures with the hash of each kernel's source file and of the",
          "shared device header, and bench.py reports roofline.traffic only while that hash matches.", ""]
    with open(os.path.join(dst, f"hbm_traffic_{key}.md"), "w") as f:
        f.write("\n".join(md + lines) + "\n")
    return res, lines, fr, wr


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def source_hash(src):
    """Hash of a kernel's source file and of the shared device header."""
    csrc = os.path.join(ROOT, "paper_2210_06713_amd", "csrc")
    return hashlib.sha256(open(os.path.join(csrc, src), "rb").read() +
                          open(os.path.join(csrc, "common.cuh"), "rb").read()).hexdigest()[:16]


SQ_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM")


def sq_summary(qdir, dst, command, title):
    """Per-kernel busy fractions from one run of shader-sequencer counters
    (median over each kernel's dispatches)."""
    per = {}
    names = {}
    for r in _rows(qdir):
        key = r.get("Dispatch_Id")
        d = per.setdefault(key, {})
        c = r.get("Counter_Name")
        d[c] = d.get(c, 0.0) + float(r["Counter_Value"])
        names[key] = r.get("Kernel_Name")
    by_kernel = {}
    for key, d in per.items():
        if "GRBM_GUI_ACTIVE" not in d or not all(c in d for c in SQ_COUNTERS):
            continue
        n = names[key].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].strip()
        cyc = d["GRBM_GUI_ACTIVE"] / N_XCD
        if cyc <= 0:
            continue
        by_kernel.setdefault(n, []).append((cyc, 100.0 * d["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * N_SIMD),
                                            100.0 * 4 * d["SQ_ACTIVE_INST_VALU"] / (cyc * N_SIMD),
                                            100.0 * 4 * d["SQ_ACTIVE_INST_LDS"] / (cyc * N_SIMD),
                                            100.0 * 4 * d["SQ_ACTIVE_INST_VMEM"] / (cyc * N_SIMD)))
    out = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
           "Per kernel, the median over its dispatches. cycles = GRBM_GUI_ACTIVE / 8 (rocprofv3 sums it",
           "over the eight XCDs); matrix cores busy = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x 1024 SIMDs);",
           "VALU / LDS issue = SQ_ACTIVE_INST_{VALU,LDS} x 4 (quad cycles) / (cycles x 1024 SIMDs).",
           "(SQ_ACTIVE_INST_VMEM reads zero for every kernel on this chip and is not shown.)",
           "", "| kernel | dispatches | cycles (median) | matrix cores busy % | VALU issue % | LDS issue % |",
           "|---|---:|---:|---:|---:|---:|"]
    for n in sorted(by_kernel):
        v = by_kernel[n]
        med = [_median([x[i] for x in v]) for i in range(5)]
        label = n if len(n) <= 60 else n[:57] + "..."
        out.append(f"| {label} | {len(v)} | {med[0]:.0f} | {med[1]:.1f} | {med[2]:.1f} | {med[3]:.1f} |")
    with open(dst, "w") as f:
        f.write("\n".join(out) + "\n")
    return out


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
    ap.add_argument("--sq-summary", nargs=4, metavar=("COUNTER_DIR", "DST_MD", "COMMAND", "TITLE"))
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="512")
    ap.add_argument("--steps", type=int, default=2)
    a = ap.parse_args()
    if a.stats_md:
        stats_markdown(*a.stats_md)
    elif a.sq_summary:
        print("\n".join(sq_summary(*a.sq_summary)))
    elif a.summarize:
        res, lines, fr, wr = summarize(*a.summarize, workload=a.workload)
        print("\n".join(lines))
        print(f"calibration: fetch x{fr:.4f}, write x{wr:.4f}")
    else:
        run(a.workload, a.steps)

#!/usr/bin/env python3
"""Benchmark of the DNA KL-NMF hot path on one MI355X.

One step = one full DNA iteration of Algorithm 1 (H half-step, step 16, W
half-step, step 29) on a synthetic workload resident in HBM.  Default workload:
N = 1024, T = 8192, R = 64 in float32 (Gamma(0.5) factors, 30%-dense planted
H0, Poisson counts at mean 5).  Prints ONE JSON line with iterations/s, the
roofline record of the dominant kernel (HIP-event timed), time-to-target-KL
against MU, and the FP64 oracle timed on the host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DNA iters/s and time-to-target-KL vs MU (N×T×R), MFMA util %, 1 MI355X"
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 matrix peak
PEAK_16_TFLOPS = 2500.0       # MI355X dense BF16 / FP16 matrix peak
PEAK_HBM_GBS = 8000.0
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}

WORKLOADS = {
    2: "Gamma(0.5) factors, 30%-dense H0, Poisson counts at mean 5",
    3: "spectrogram-like smooth Gamma-bump bases, Gamma(0.3) activations, Poisson mean 2",
    4: "Dirichlet(0.05) bases, Gamma(1,20) activations, ~95% zero counts stored dense",
}


def kernel_work(name, N, T, R):
    """Algorithmic work of one launch of each kernel: (kind, amount).

    The paper's count is four O(NRT) products per half-step: A and B (the
    gradient/Hessian kernels, 2 x 2NRT) and the two candidate reconstructions
    (the cost kernels, 2 x 2NRT).  The ratio kernels recompute Z = W H (2NRT),
    which the paper carries over instead; it is reported but is not algorithmic.
    """
    nrt = float(N) * R * T
    table = {}
    for sfx in ("", "16"):
        table.update({
            f"gh{sfx}_H": ("flops", 4 * nrt), f"gh{sfx}_W": ("flops", 4 * nrt),
            f"cost{sfx}_H": ("flops", 4 * nrt), f"cost{sfx}_W": ("flops", 4 * nrt),
            f"ratio{sfx}_H": ("flops_recompute", 2 * nrt), f"ratio{sfx}_W": ("flops_recompute", 2 * nrt),
        })
    table["qmax16"] = ("flops_recompute", 2 * nrt)
    # fused kernels (R <= 64): Z recompute + gradient products / the two reconstructions
    table["rgh_H"] = table["rgh_W"] = ("flops", 4 * nrt)
    table["costf_H"] = table["costf_W"] = ("flops", 4 * nrt)
    # the one-kernel H half-step: gradient products and the two reconstructions
    table["hstep_cols"] = ("flops", 8 * nrt)
    return table.get(name)


def _unmangle(name):
    """(base, template arguments) of a mangled dna:: kernel name, which rocprofv3
    leaves mangled when a template argument is a 16-bit float type; None if the
    name is not of that form."""
    import re
    m = re.match(r"_ZN3dna(\d+)", name)
    if not m:
        return None
    n = int(m.group(1))
    rest = name[m.end():]
    base, rest = rest[:n], rest[n:]
    if not rest.startswith("I"):
        return base, []
    parts = []
    for tok in re.findall(r"L[ib]\d+E|DF16[b_]", rest[1:rest.find("EEv") + 1]):
        if tok.startswith("DF16"):
            parts.append("bf16" if tok == "DF16b" else "fp16")
        elif tok.startswith("Lb"):
            parts.append("true" if tok[2:-1] == "1" else "false")
        else:
            parts.append(tok[2:-1])
    return base, parts


def kernel_key(rocprof_name):
    """Bench kernel key of a rocprofv3 kernel name (the names prof_begin uses)."""
    import re
    um = _unmangle(rocprof_name.strip())
    if um is not None:
        base, parts = um
        nm = base + ("<" + ", ".join(parts) + ">" if parts else "")
    else:
        nm = rocprof_name.split("(")[0].replace("void ", "").replace("dna::", "")
    base = re.sub(r"<.*>", "", nm)
    base = {"k_gh2_H": "k_gh_H", "k_gh2_W": "k_gh_W"}.get(base, base)   # both gradient forms profile as gh_H/W
    targs = re.search(r"<(.*)>", nm)
    side = None
    if targs:
        parts = [t.strip() for t in targs.group(1).split(",")]
        if base in ("k_gh16", "k_cost16") and len(parts) >= 2:
            side = parts[1]
        if base == "k_ratio16" and len(parts) >= 3:
            side, maxonly = parts[1], parts[2]
            if maxonly == "true":
                return "qmax16"
        if base == "k_ratio":
            return {"0": "ratio_H", "1": "ratio_W", "8": "ratio_H", "9": "ratio_W"}.get(parts[0], "ratio_" + parts[0])
        if base in ("k_sp_grad", "k_sp_cost", "k_sp_comb", "k_sp_cost_comb"):
            mu = "_mu" if base == "k_sp_grad" and parts[-1] == "true" else ""
            return base[2:] + mu + ("_H" if parts[0] == "0" else "_W")
    if side is not None:
        return base[2:] + ("_H" if side == "0" else "_W")
    return base[2:] if base.startswith("k_") else base


def strip_comments(src):
    """C/C++ source text without its comments and blank runs (string and character
    literals kept as they are), so that editing a comment changes no hash."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "\n".join(" ".join(l.split()) for l in "".join(out).splitlines() if l.strip())


def source_hash():
    """Hash of the HIP sources' code (comments left out): traffic counters are only valid for the
    build they were taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_1301_3389_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), encoding="utf-8") as fh:
                h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_summary(args):
    """Write profiles/traffic_<tag>.json from four rocprofv3 --pmc output folders: FETCH_SIZE and
    WRITE_SIZE of the benchmark, and of the plain copy (--copy-calibration) that scales them."""
    import csv
    import glob

    def per_kernel(folder, counter):
        f = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)[0]
        acc = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write, cfetch, cwrite = args.traffic_summary
    copy_bytes = 256 * 1024 * 1024
    cf = max(v for k, v in per_kernel(cfetch, "FETCH_SIZE").items() if "copy" in k.lower())
    cw = max(v for k, v in per_kernel(cwrite, "WRITE_SIZE").items() if "copy" in k.lower())
    out = {"source_hash": source_hash(), "unit": "bytes per dispatch",
           "fetch_scale": copy_bytes / (cf * 1024), "write_scale": copy_bytes / (cw * 1024),
           "copy_fetch_kib": cf, "copy_write_kib": cw, "kernels": {}}
    fk, wk = per_kernel(fetch, "FETCH_SIZE"), per_kernel(write, "WRITE_SIZE")
    for k in sorted(set(fk) & set(wk)):
        out["kernels"][k] = {"fetch_kib": fk[k], "write_kib": wk[k],
                             "bytes": fk[k] * 1024 * out["fetch_scale"] + wk[k] * 1024 * out["write_scale"]}
    path = os.path.join(ROOT, "profiles", f"traffic_{args.traffic_tag}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


def traffic_of(kernel, tag):
    """Measured HBM bytes per launch of `kernel` from profiles/traffic_<tag>.json, or None when
    the file is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["bytes"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4])
    ap.add_argument("--sparse", default=None, choices=["tdt2", "newsgroup"],
                    help="sparse-V workload shaped like a Sec. 4.2 matrix instead of a dense config")
    ap.add_argument("--rank", type=int, default=40, help="R of the sparse workload")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="per-iteration MU / MU+cost / DNA times at the paper's dense shapes (Table 1)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="bound on the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-target", action="store_true", help="skip the time-to-target-KL runs")
    ap.add_argument("--mu-iters", type=int, default=1000, help="MU iterations that fix the target KL")
    ap.add_argument("--dna-iters", type=int, default=1000, help="DNA iteration budget for the target")
    ap.add_argument("--gemm", default="fp32", choices=["fp32", "bf16", "fp16"],
                    help="operand type of the DNA matrix products (16-bit: FP32 accumulate, FP64 sums)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (HBM counter calibration)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write profiles/traffic_<tag>.json from four rocprofv3 --pmc output folders")
    ap.add_argument("--traffic-tag", default=None, help="tag of the traffic file (default: workload tag)")
    ap.add_argument("--rho", type=float, default=0.0,
                    help="eq. 2 weight of sum W (with --lam: time the regularised iteration; "
                         "no time-to-target or CPU leg)")
    ap.add_argument("--lam", type=float, default=0.0, help="eq. 2 weight of sum H")
    ap.add_argument("--streams", type=int, default=4,
                    help="--paper-sweep: also time this many independent problems on as many streams")
    ap.add_argument("--unrolled", action="store_true",
                    help="time the differentiable unrolled H-solve (N=513 R=1024 T=4096, K=20): forward + backward")
    ap.add_argument("--no-r512", action="store_true",
                    help="skip the R = 512 records (N=4096 T=32768, FP32 and BF16) of the default run")
    return ap.parse_args()


def workload_tag(config, gemm):
    return f"config{config}_{gemm}"


def copy_calibration():
    """A plain copy kernel of known size: 256 MiB read + 256 MiB written per launch."""
    import torch
    n = 64 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))


def timed_steps(dna, V, W, H, steps, gemm, **kw):
    import torch
    dna.iterate(V, W, H, 2, gemm=gemm, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dna.iterate(V, W, H, steps, gemm=gemm, **kw)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def iters_to_targets(dna, V, W0, H0, targets, budget, gemm, chunk=10, **kw):
    """DNA iterations (from the same start, step 1 first) until the KL is at or
    below each of `targets`; the KL after every iteration is recorded on the
    device and checked every `chunk` iterations.  Returns ({target: first
    iteration or None}, last KL)."""
    import numpy as np
    import torch
    W, H = W0.clone(), H0.clone()
    dna.normalize(0, W, H)
    kls = torch.empty(budget + 1, dtype=torch.float64, device=V.device)
    dna.kl_cost(V, W, H, out=kls[0:1])
    done = 0
    hits = {t: None for t in targets}
    while done < budget:
        m = min(chunk, budget - done)
        for k in range(m):
            dna.iterate(V, W, H, 1, gemm=gemm, **kw)
            dna.kl_cost(V, W, H, out=kls[done + k + 1:done + k + 2])
        done += m
        host = kls[:done + 1].cpu().numpy()
        for t in targets:
            if hits[t] is None:
                h = np.nonzero(host <= t)[0]
                if h.size:
                    hits[t] = int(h[0])
        if all(v is not None for v in hits.values()):
            break
    return hits, float(kls[done].item())


def mu_reference(dna, V, W0, H0, marks):
    """MU (no cost) from the same start, step 1 first: the KL after each of the
    iteration counts in `marks` (ascending) and the ms per MU iteration."""
    import torch
    W, H = W0.clone(), H0.clone()
    dna.normalize(0, W, H)
    kl, done, wall = {}, 0, 0.0
    for m in marks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dna.mu_iterate(V, W, H, m - done, with_cost=False)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        done = m
        kl[m] = dna.kl_cost(V, W, H).item()
    return kl, 1e3 * wall / marks[-1]


def cpu_baseline(w, seconds):
    """The FP64 oracle, as it stands, on the host: full DNA iterations of the same
    workload until about `seconds` of CPU work (at least one)."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = int(os.environ.get("OMP_NUM_THREADS", "1"))
    V = w.V.astype(np.float64)
    Wc, Hc = oracle.normalize_w_columns(w.W, w.H)
    t0 = time.perf_counter()
    n = 0
    while True:
        Hc = oracle.h_step(V, Wc, Hc).X
        Wc, Hc = oracle.normalize_h_rows(Wc, Hc)
        Wc = oracle.w_step(V, Wc, Hc).X
        Wc, Hc = oracle.normalize_w_columns(Wc, Hc)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    out = {"value": n / dt, "unit": "DNA iterations/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{n} full DNA iterations (FP64 NumPy) of the same workload from the same initial state",
           "cpu_model": cpu_model()}
    try:                                   # the same oracle on one thread
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            W1, H1 = oracle.normalize_w_columns(w.W, w.H)
            t1 = time.perf_counter()
            n1 = 0
            while True:
                H1 = oracle.h_step(V, W1, H1).X
                W1, H1 = oracle.normalize_h_rows(W1, H1)
                W1 = oracle.w_step(V, W1, H1).X
                W1, H1 = oracle.normalize_w_columns(W1, H1)
                n1 += 1
                if time.perf_counter() - t1 >= seconds:
                    break
            out["single_thread"] = {"value": n1 / (time.perf_counter() - t1), "cores": 1,
                                    "sample": f"{n1} full DNA iterations on one thread"}
    except ImportError:  # pragma: no cover
        pass
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return None


def sparse_kernel_bytes(name, N, T, R, nnz, nseg_r, nseg_c):
    """Algorithmic HBM bytes of one launch of a sparse-V kernel: the index and
    value streams it must read, the factor rows it gathers counted once, and
    what it writes (segment tables and small vectors left out)."""
    f = 4.0
    table = {
        "sp_zq": 12 * nnz + f * R * (N + T) + 8 * nnz,                 # row, col, val; W, H^t; q, q-bar
        "sp_grad_H": 20 * nnz + f * N * R + 16 * nseg_c * R,            # pos, row, q, q-bar, val; W; partials
        "sp_grad_W": 16 * nnz + f * T * R + 16 * nseg_r * R,            # col, q, q-bar, val; H^t; partials
        "sp_cost_H": 16 * nnz + f * N * R + 2 * f * T * R,              # pos, row, col, val; W; candidates^t
        "sp_cost_W": 16 * nnz + f * T * R + 2 * f * N * R,              # row, col, val (+pos); H^t; candidates
    }
    return table.get(name)


def sparse_main(args):
    """One JSON line for a sparse-V workload (Sec. 4.2 shapes): DNA iterations/s,
    the dominant kernel against the HBM roofline, and the time to MU's KL."""
    import torch
    from paper_1301_3389_amd import dna, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    rows, cols, vals, N, T, W0n, H0n = synth.sparse_workload(args.sparse, R=args.rank)
    R = args.rank
    sv = dna.SparseV(rows, cols, vals, N, T, device=dev)
    W0, H0 = torch.from_numpy(W0n).to(dev), torch.from_numpy(H0n).to(dev)
    W, H = W0.clone(), H0.clone()
    dna.normalize(0, W, H)
    dna.sparse_iterate(sv, W, H, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dna.sparse_iterate(sv, W, H, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    dna.profile_reset()
    dna.profile_enable(True)
    dna.sparse_iterate(sv, W, H, args.steps)
    torch.cuda.synchronize()
    stats = dna.profile_read()
    dna.profile_enable(False)
    kernels = {k: {"launches": n, "avg_ms": t / max(n, 1), "total_ms": t} for k, (n, t) in stats.items()}
    nseg_r, nseg_c = sv.c.nseg_r, sv.c.nseg_c
    cands = {k: v for k, v in kernels.items() if sparse_kernel_bytes(k, N, T, R, sv.nnz, nseg_r, nseg_c)}
    dom = max(cands, key=lambda k: cands[k]["total_ms"])
    nbytes = sparse_kernel_bytes(dom, N, T, R, sv.nnz, nseg_r, nseg_c)
    achieved = nbytes / (cands[dom]["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "avg_ms": cands[dom]["avg_ms"], "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": traffic_of(dom, "sparse_" + args.sparse)}
    if roofline["traffic"] is not None:
        roofline["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    target = None
    if not args.no_target:
        Wm, Hm = W0.clone(), H0.clone()
        dna.normalize(0, Wm, Hm)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        dna.sparse_mu_iterate(sv, Wm, Hm, args.mu_iters)
        torch.cuda.synchronize()
        mu_wall = time.perf_counter() - tm
        kl_target = dna.sparse_kl_cost(sv, Wm, Hm).item()
        Wd, Hd = W0.clone(), H0.clone()
        kls = dna.sparse_fit(sv, Wd, Hd, args.dna_iters, record_kl=True).cpu().numpy()
        hit = [k for k, x in enumerate(kls) if x <= kl_target]
        k_hit = hit[0] if hit else None
        target = {"target_kl": kl_target, "mu_iters": args.mu_iters,
                  "mu_ms_per_iter": 1e3 * mu_wall / args.mu_iters, "mu_time_to_target_s": mu_wall,
                  "dna_ms_per_iter": ms, "dna_iters_to_target": k_hit,
                  "dna_time_to_target_s": k_hit * ms / 1e3 if k_hit is not None else None,
                  "kl_at_stop": float(kls[k_hit] if k_hit is not None else kls[-1])}
        if k_hit:
            target["speedup_vs_mu"] = mu_wall / (k_hit * ms / 1e3)
    shape = {"tdt2": "TDT2", "newsgroup": "Newsgroup"}[args.sparse]
    out = {
        "metric": "DNA iterations/s, sparse V", "value": args.steps / wall, "unit": "DNA iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "accumulate": "f32 sums, f64 cost and selection sums",
        "data": "synthetic",
        "config": {"workload": f"sparse term-document counts shaped like {shape} ({N} x {T}, "
                               f"{sv.nnz / (N * T) * 100:.2f}% nonzeros, Zipf row lengths), R={R}",
                   "N": N, "T": T, "R": R, "nnz": sv.nnz, "parallelism": "single GPU"},
        "roofline": roofline, "kernels": kernels, "time_to_target": target,
    }
    print(json.dumps(out))


def unrolled_main(args):
    """The differentiable unrolled H-solve at its workload (W fixed 513 x 1024,
    V = Poisson(W H0) with T = 4096 columns, K = 20 DNA H-updates, loss
    ||H_K - H0||^2): ms per forward (K updates with checkpoints) and per
    backward (the hand-written adjoint), per-kernel HIP-event times of each,
    and the roofline record of the dominant algorithmic kernel of each.
    Algorithmic work: forward 8NRT per update (the paper's four products);
    backward 12NRT per update (qbar, qbbar: 4NRT in zbar; the three W-gradient
    products: 6NRT in wbar; W^t zbar: 2NRT).  The forward keeps Z, Q, Q-bar and
    the gradient sums of every update for the backward (the autograd path's
    calls), so the backward recomputes no product."""
    import torch
    from paper_1301_3389_amd import dna, synth
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    K = 20
    w = synth.config5()
    N, T = w.V.shape
    R = w.W.shape[1]
    V = torch.from_numpy(w.V).to(dev)
    W = torch.from_numpy(w.W).to(dev)
    H = torch.from_numpy(w.H).to(dev)
    H0 = torch.from_numpy(w.H0).to(dev)
    nrt = float(N) * R * T

    # the autograd path's calls: the forward keeps Z, Q, Q-bar and the gradient
    # sums of every update, which the backward reads instead of recomputing
    def fwd():
        return dna.unrolled_forward(V, W, H, K, keep_sums=True)

    def bwd(Hc, sel, aux):
        return dna.unrolled_backward(V, W, Hc, sel, K, 2.0 * (Hc[K] - H0).contiguous(), aux=aux)

    for _ in range(max(1, args.warmup)):
        Hc, sel, aux = fwd()
        bwd(Hc, sel, aux)
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        Hc, sel, aux = fwd()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        bwd(Hc, sel, aux)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd_ms, bwd_ms = 1e3 * (t1 - t0) / reps, 1e3 * (t2 - t1) / reps

    def kernel_profile(fn):
        dna.profile_reset()
        dna.profile_enable(True)
        fn()
        torch.cuda.synchronize()
        st = dna.profile_read()
        dna.profile_enable(False)
        return {k: {"launches": n, "avg_ms": ms / max(n, 1), "total_ms": ms} for k, (n, ms) in st.items()}

    kf = kernel_profile(fwd)
    kb = kernel_profile(lambda: bwd(Hc, sel, aux))
    peak = PEAK_FP32_TFLOPS

    def roof(kernels, work):
        cand = {k: v for k, v in kernels.items() if k in work}
        dom = max(cand, key=lambda k: cand[k]["total_ms"])
        ach = work[dom] / (cand[dom]["avg_ms"] * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": dom, "avg_ms": cand[dom]["avg_ms"], "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None}
    fwd_work = {"gh_H": 4 * nrt, "cost_H": 4 * nrt}
    bwd_work = {"zbar": 4 * nrt, "wbar": 6 * nrt, "gh_mu_H": 2 * nrt}
    alg_f, alg_b = K * 8 * nrt, K * 12 * nrt
    out = {"metric": "unrolled DNA H-solve, forward + backward per second", "value": 1e3 / (fwd_ms + bwd_ms),
           "unit": "forward+backward/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
           "ms_per_step": fwd_ms + bwd_ms, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"unrolled H-solve, W fixed Gamma(0.5) {N} x {R}, V = Poisson(W H0) with "
                                  f"T={T}, K={K} DNA H-updates, loss ||H_K - H0||^2", "N": N, "T": T, "R": R, "K": K,
                      "kept_sums": aux is not None, "parallelism": "single GPU"},
           "forward_ms": fwd_ms, "backward_ms": bwd_ms,
           "forward_tflops_algorithmic": alg_f / (fwd_ms * 1e-3) / 1e12,
           "backward_tflops_algorithmic": alg_b / (bwd_ms * 1e-3) / 1e12,
           "roofline": roof(kb, bwd_work), "roofline_forward": roof(kf, fwd_work),
           "kernels_forward": kf, "kernels_backward": kb}
    print(json.dumps(out))


def paper_sweep(args):
    """Table 1 of the paper at its dense shapes (ORL 4096 x 165, PIE 1024 x 11554;
    R = 10, 20, 40, 80) with synthetic data of those shapes: ms per iteration of
    MU without cost, MU with cost and DNA, and the DNA iterations needed to reach
    the KL of 500 MU iterations (the paper's Fig. 1 comparison)."""
    import torch
    from paper_1301_3389_amd import dna, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def per_iter(step, W, H, k):
        step(W, H, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(W, H, k)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / k

    def concurrent(V, W, H, S, k):
        """ms per problem-iteration with S independent problems, one per stream
        (default priority), their iterations issued in turn; each stream has its
        own workspace."""
        streams = [torch.cuda.Stream() for _ in range(S)]
        Ws, Hs = [W.clone() for _ in range(S)], [H.clone() for _ in range(S)]
        for st, a, b in zip(streams, Ws, Hs):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                dna.iterate(V, a, b, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            for st, a, b in zip(streams, Ws, Hs):
                with torch.cuda.stream(st):
                    dna.iterate(V, a, b, 1)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / (k * S)

    rows = []
    for name in ("orl", "pie"):
        for R in (10, 20, 40, 80):
            w = synth.paper_dense(name, R)
            V = torch.from_numpy(w.V).to(dev)
            W0, H0 = torch.from_numpy(w.W).to(dev), torch.from_numpy(w.H).to(dev)
            W, H = W0.clone(), H0.clone()
            dna.normalize(0, W, H)
            k = args.steps

            def mu(Wx, Hx, n, cost):
                dna.mu_iterate(V, Wx, Hx, n, with_cost=cost)
            mu_ms = per_iter(lambda a, b, n: mu(a, b, n, False), W.clone(), H.clone(), k)
            muc_ms = per_iter(lambda a, b, n: mu(a, b, n, True), W.clone(), H.clone(), k)
            dna_ms = per_iter(lambda a, b, n: dna.iterate(V, a, b, n), W.clone(), H.clone(), k)
            dna_ms_conc = concurrent(V, W, H, args.streams, k) if args.streams > 1 else None
            Wm, Hm = W.clone(), H.clone()
            mu(Wm, Hm, 500, False)
            target = dna.kl_cost(V, Wm, Hm).item()
            Wd, Hd = W0.clone(), H0.clone()
            kls = dna.fit(V, Wd, Hd, 500, record_kl=True).cpu().numpy()
            hit = [i for i, x in enumerate(kls) if x <= target]
            rows.append({"dataset": name, "N": w.V.shape[0], "T": w.V.shape[1], "R": R,
                         "mu_ms": mu_ms, "mu_cost_ms": muc_ms, "dna_ms": dna_ms,
                         "dna_over_mu_cost": dna_ms / muc_ms, "mu_cost_over_mu": muc_ms / mu_ms,
                         "streams": args.streams, "dna_ms_per_problem_concurrent": dna_ms_conc,
                         "dna_iters_to_mu500_kl": hit[0] if hit else None})
    out = {"metric": "ms per iteration at the paper's dense shapes (Table 1)", "unit": "ms",
           "n_gpus": 1, "steps": args.steps, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "ORL-shaped 4096 x 165 and PIE-shaped 1024 x 11554 Poisson counts of a "
                                  "Gamma(0.5) product at mean 60, R = 10, 20, 40, 80",
                      "parallelism": "single GPU"},
           "sweep": rows}
    print(json.dumps(out))


def main():
    args = parse()
    if args.paper_sweep:
        paper_sweep(args)
        return
    if args.unrolled:
        unrolled_main(args)
        return
    if args.sparse:
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        sparse_main(args)
        return
    if args.traffic_tag is None:
        args.traffic_tag = workload_tag(args.config, args.gemm)
    if args.traffic_summary:
        traffic_summary(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(with V sharded by columns, the H half-step is local and the W half-step "
              "needs one all-reduce of its N x R gradient sums and per-row costs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1301_3389_amd import dna, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = synth.config(args.config)
    N, T = w.V.shape
    R = w.W.shape[1]
    V = torch.from_numpy(w.V).to(dev)
    W0 = torch.from_numpy(w.W).to(dev)
    H0 = torch.from_numpy(w.H).to(dev)

    gemm = args.gemm
    reg = dict(rho=args.rho, lam=args.lam)
    regularised = args.rho > 0 or args.lam > 0
    if regularised:
        args.no_target = args.no_cpu_baseline = True
    rec = dense_record(dna, V, W0, H0, gemm, args.steps, args.warmup, args.traffic_tag, reg)

    # ---- time to target KL (MU's KL after --mu-iters iterations) ----------
    target = None
    if not args.no_target:
        kl_mu, mu_ms = mu_reference(dna, V, W0, H0, [args.mu_iters])
        kl_target = kl_mu[args.mu_iters]
        Wc, Hc = W0.clone(), H0.clone()
        dna.normalize(0, Wc, Hc)
        nc = min(100, args.mu_iters)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        dna.mu_iterate(V, Wc, Hc, nc, with_cost=True)
        torch.cuda.synchronize()
        mu_cost_ms = 1e3 * (time.perf_counter() - tc) / nc
        mu_wall = mu_ms * args.mu_iters / 1e3
        target = {"target_kl": kl_target, "mu_iters": args.mu_iters,
                  "mu_ms_per_iter_no_cost": mu_ms,
                  "mu_ms_per_iter_with_cost": mu_cost_ms, "mu_time_to_target_s": mu_wall,
                  "dna_iter_budget": args.dna_iters}
        forms = [gemm] + (["fp32"] if gemm != "fp32" else [])
        for g in forms:
            ms = rec["ms_per_step"] if g == gemm else timed_steps(dna, V, W0.clone(), H0.clone(), 20, g)
            hits, kl_last = iters_to_targets(dna, V, W0, H0, [kl_target], args.dna_iters, g)
            k_hit = hits[kl_target]
            r = {"ms_per_iter": ms, "iters_to_target": k_hit,
                 "time_to_target_s": (k_hit * ms / 1e3) if k_hit is not None else None,
                 "kl_at_stop": kl_last}
            if k_hit:
                r["speedup_vs_mu_no_cost"] = mu_wall / (k_hit * ms / 1e3)
            target[f"dna_{g}"] = r
        if R <= 64 and gemm == "fp32":
            # the damped selection (Newton costed alone, kept iff it does not raise the cost)
            ms = timed_steps(dna, V, W0.clone(), H0.clone(), args.steps, "fp32", select="newton_first")
            hits, kl_last = iters_to_targets(dna, V, W0, H0, [kl_target], args.dna_iters, "fp32",
                                             select="newton_first")
            k_hit = hits[kl_target]
            r = {"ms_per_iter": ms, "iters_to_target": k_hit,
                 "time_to_target_s": (k_hit * ms / 1e3) if k_hit is not None else None, "kl_at_stop": kl_last}
            if k_hit:
                r["speedup_vs_mu_no_cost"] = mu_wall / (k_hit * ms / 1e3)
            target["dna_fp32_newton_first"] = r

    out = {
        "metric": METRIC, "value": rec["value"], "unit": "DNA iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[gemm],
        "accumulate": "f32 products, f64 cost and selection sums",
        "data": "synthetic",
        "config": {"workload": f"DNA KL-NMF, N={N} T={T} R={R}, {WORKLOADS[args.config]}",
                   "N": N, "T": T, "R": R, "iteration": "H step, step 16, W step, step 29",
                   "parallelism": "single GPU", **({"rho": args.rho, "lambda": args.lam} if regularised else {})},
        **{k: rec[k] for k in ("gpu_ms_per_step", "algorithmic_gflops", "mfma_frac_algorithmic", "roofline",
                               "kernels", "profiled_ms_per_step")},
        "time_to_target": target,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    del V, W0, H0
    if args.config == 2 and not args.no_r512 and not regularised:
        torch.cuda.empty_cache()
        out["r512"] = r512_records(dna, synth, dev, args)
    print(json.dumps(out))


def dense_record(dna, V, W0, H0, gemm, steps, warmup, traffic_tag, reg=None):
    """Timed DNA iterations (one dna_iterate call of `steps` iterations after
    `warmup` untimed ones, step 1 first) and the per-kernel HIP-event times of
    a repeat of the same call; the roofline record of the dominant flops kernel."""
    import torch
    reg = reg or {}
    N, T = V.shape
    R = W0.shape[1]
    W, H = W0.clone(), H0.clone()
    dna.normalize(0, W, H, **reg)                            # Algorithm 1 step 1
    dna.iterate(V, W, H, warmup, gemm=gemm, **reg)
    torch.cuda.synchronize()
    # ---- timed region -----------------------------------------------------
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    dna.iterate(V, W, H, steps, gemm=gemm, **reg)            # `steps` full iterations, one call
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    # ---- per-kernel HIP-event timing over a repeat of the timed region ---
    dna.profile_reset()
    dna.profile_enable(True)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    dna.iterate(V, W, H, steps, gemm=gemm, **reg)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    stats = dna.profile_read()
    dna.profile_enable(False)
    kernels = {k: {"launches": n, "avg_ms": ms / max(n, 1), "total_ms": ms} for k, (n, ms) in stats.items()}
    ranked = sorted(((k, v) for k, v in kernels.items() if kernel_work(k, N, T, R)
                     and kernel_work(k, N, T, R)[0] == "flops"), key=lambda kv: -kv[1]["total_ms"])
    dom, krec = ranked[0]
    flops = kernel_work(dom, N, T, R)[1]
    achieved = flops / (krec["avg_ms"] * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if gemm == "fp32" else PEAK_16_TFLOPS
    roofline = {"bound": "mfma", "kernel": dom, "avg_ms": krec["avg_ms"], "achieved": achieved,
                "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic_of(dom, traffic_tag)}
    if roofline["traffic"] is not None:
        roofline["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    value = steps / wall
    gflops = 16.0 * N * R * T * value / 1e9
    return {"value": value, "ms_per_step": 1e3 * wall / steps, "gpu_ms_per_step": gpu_ms / steps,
            "algorithmic_gflops": gflops, "mfma_frac_algorithmic": gflops / 1e3 / peak,
            "roofline": roofline, "kernels": kernels, "profiled_ms_per_step": 1e3 * prof_wall / steps}


def r512_records(dna, synth, dev, args):
    """The high-rank workload (N=4096 T=32768 R=512, spectrogram-like) in the
    plain FP32 form and the BF16 precision form: iterations/s, the dominant
    kernel's roofline record, and the time to MU's KL after 200 and after 1000
    iterations from the same start."""
    import torch
    w = synth.config3()
    N, T = w.V.shape
    R = w.W.shape[1]
    V = torch.from_numpy(w.V).to(dev)
    W0 = torch.from_numpy(w.W).to(dev)
    H0 = torch.from_numpy(w.H).to(dev)
    del w
    out = {"config": {"workload": f"DNA KL-NMF, N={N} T={T} R={R}, {WORKLOADS[3]}", "N": N, "T": T, "R": R},
           "steps": args.steps, "warmup": args.warmup}
    for g in ("fp32", "bf16"):
        rec = dense_record(dna, V, W0, H0, g, args.steps, args.warmup, workload_tag(3, g))
        rec["kernels"] = {k: v for k, v in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["total_ms"])[:8]}
        rec["dtype"] = DTYPE[g]
        out[g] = rec
    if not args.no_target:
        marks = [200, 1000]
        kl_mu, mu_ms = mu_reference(dna, V, W0, H0, marks)
        tt = {"mu_ms_per_iter": mu_ms, "target_kl": {str(m): kl_mu[m] for m in marks},
              "mu_time_to_target_s": {str(m): m * mu_ms / 1e3 for m in marks}}
        for g in ("fp32", "bf16"):
            hits, kl_last = iters_to_targets(dna, V, W0, H0, [kl_mu[m] for m in marks], args.dna_iters, g)
            ms = out[g]["ms_per_step"]
            r = {"ms_per_iter": ms, "kl_at_stop": kl_last}
            for m in marks:
                k = hits[kl_mu[m]]
                r[f"iters_to_mu{m}"] = k
                r[f"time_to_mu{m}_s"] = k * ms / 1e3 if k is not None else None
                if k:
                    r[f"speedup_vs_mu{m}"] = (m * mu_ms) / (k * ms)
            tt[f"dna_{g}"] = r
        out["time_to_target"] = tt
    return out


if __name__ == "__main__":
    main()

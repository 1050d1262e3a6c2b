"""Benchmark: candidate merges evaluated per second on one MI355X.

Workload: 256 FP32 blocks of 1024 x 256 in 16 groups (shared 1024 x 32 bases rotated
per block by principal angles ~U(0, 0.3)), rank r = 64, all 32,640 anchor-first pairs
in one batched evaluation.  One step = one cmsvd_merge_errors call over all pairs:
block norms and Grams, anchor initialisation (rank-64 truncated SVD of every anchor),
projections (FP32 operands on the FP32 matrix cores by default, --projection), core
eigenvalues and plug-in errors (FP64).  Inputs are resident in HBM before the timed
region.  The same steps are then replayed from a captured HIP graph (the `graph` field,
capture time apart).

Also reported on the same GPU: the plain per-pair method (one cmsvd_merge_errors call
per pair, serialised, no reuse across pairs), the same per-pair math in library form
(torch FP64 SVDs, for context), the roofline position of the dominant
stage (timed with HIP events on the library's stream during the timed steps), the FP64
CPU oracle timed on a bounded sample of the same pairs, and the deviation of the GPU
results from the oracle on that sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "candidate merges evaluated/sec (batched vs plain, same GPU) at ≤1e-5 rel error"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 (vector and matrix), 256 CU x 2.4 GHz
# dense matrix-core peaks of MI355X per projection operand type, and the kernel name
PROJ_PEAK = {"f64": (78.6, "gemm_f64_kernel (Y = U^T B)"), "f32": (157.3, "gemm_f32_wide_kernel (Y = U^T B)"),
             "bf16": (2500.0, "gemm_bf16_kernel (Y = U^T B, one BF16 pass)"),
             "bf16x3": (2500.0, "gemm_bf16_kernel (Y = U^T B, three BF16 passes)")}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CPU_SHARE_PER_GPU = 16


def host_cpus():
    """The host cores the CPU oracle runs on: the process's affinity set, bounded by the
    job's share of the host (the cgroup CPU quota when one is set, else the 16 host cores
    that the GPU hosts give each GPU), with the machine's logical CPU count and model for
    the record."""
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        affinity = os.cpu_count() or 1
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) // int(per)))
    except (OSError, ValueError):
        pass
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = min(affinity, quota if quota else CPU_SHARE_PER_GPU)
    return {"threads": max(1, threads), "affinity": affinity, "cgroup_quota": quota,
            "host_logical_cpus": os.cpu_count(), "model": model}


def kernel_source_hash():
    import hashlib

    hs = hashlib.sha256()
    for name in ("eig.hip", "common.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2601_11626_amd", "csrc", name), "rb") as f:
            hs.update(f.read())
    return hs.hexdigest()[:16]


def measured_traffic(kernel, npairs):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy of known size), or None when the summary is missing
    or was taken on different kernel sources or another launch size."""
    path = os.path.join(ROOT, "profiles", "traffic_sym_eig_rotated_groups_256x1024x256_r64.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_hash") != kernel_source_hash() or rec.get("pairs") != npairs:
        return None
    return rec.get("bytes_per_launch")


def _pmc_rows(path):
    import csv

    rows = {}
    with open(path, newline="") as f:
        for rec in csv.DictReader(f):
            low = {k.lower(): v for k, v in rec.items()}
            key = (low.get("dispatch_id"), low.get("kernel_name"))
            rows[key] = rows.get(key, 0.0) + float(low.get("counter_value", 0.0))
    return rows  # (dispatch, kernel) -> counter summed over its instances (KiB)


# the headline's dominant launch: the register-resident tridiagonalisation of the split
# evaluation (n = 320: 10 tile rows of 32), whose bisection runs in tri_bisect_kernel
EIG_KERNEL = "sym_eig_reg_kernel<2, 512, 5, 5, 10, true>"
# the kernels that finish cores of order 193..320 on their trailing matrices: four waves
# from order 192 down to 160 (register and LDS tiles) and down to 64 (register tiles),
# then one wave per problem
TAIL_KERNELS = ("sym_eig_reg_kernel<2, 256, 4, 3, 6, true> (192 -> 160)",
                "sym_eig_reg_kernel<2, 256, 4, 0, 5, true> (160 -> 64)", "sym_eig_small_kernel<2, 64> (64)")
TAIL_ORDER = 192


def pmc_summary(fetch_csv, write_csv, copy_mib, kernel=EIG_KERNEL):
    """Per-launch HBM bytes of `kernel` from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for the reference copy of copy_mib MiB."""
    out = {"kernel": kernel, "copy_mib": copy_mib}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _pmc_rows(path)
        cal = [v for (d, k), v in rows.items() if "MulFunctor" in (k or "")]
        ker = [v for (d, k), v in rows.items() if kernel in (k or "")]
        if not cal or not ker:
            raise SystemExit(f"{path}: calibration dispatches {len(cal)}, {kernel} dispatches {len(ker)}")
        scale = (copy_mib << 20) / (sum(cal) / len(cal) * 1024.0)
        out[tag] = {"kib_per_launch": sum(ker) / len(ker), "launches": len(ker),
                    "copy_kib": sum(cal) / len(cal), "scale": scale,
                    "bytes_per_launch": sum(ker) / len(ker) * 1024.0 * scale}
    out["bytes_per_launch"] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    out["source_hash"] = kernel_source_hash()
    return out


def chain_grad(args, cm, workloads, torch):
    """Tail energy f = E~^2 of a 64-block chain (2048 x 512 FP32 blocks sharing a
    2048 x 96 subspace, noise 0.05, r = 128) and its gradient with respect to every
    block.  One step = one forward + backward (cmsvd_tail_energy_grad).  Checks that
    hold at any size: the Euler identity sum <grad_t, A_t> = 2 f and central
    differences of the GPU forward along random unit directions; reported (not a
    criterion): cosine and relative difference against the exact-SVD gradient 2(M - M_r)."""
    r = 128
    t0 = time.time()
    blocks_np = workloads.shared_chain(seed=0)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    log(f"generated {len(blocks)} blocks {tuple(blocks[0].shape)} in {time.time() - t0:.1f}s")
    ck = 8
    for w in range(args.warmup):
        f, grads, gap = cm.cmsvd_tail_energy_grad(blocks, r, ck)
        log(f"warmup {w + 1}/{args.warmup}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        f, grads, gap = cm.cmsvd_tail_energy_grad(blocks, r, ck)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    t2 = time.perf_counter()
    f_fwd, _, _ = cm.cmsvd_tail_energy_grad(blocks, r, ck, want_grad=False)
    torch.cuda.synchronize()
    fwd_s = time.perf_counter() - t2
    if args.no_check:
        print(json.dumps({"ms_per_step": round(1000.0 * el / max(args.steps, 1), 3),
                          "forward_only_ms": round(1000.0 * fwd_s, 3), "f": f}), flush=True)
        return
    # checks that hold at any size
    euler = sum(float(torch.sum(g * b.double())) for g, b in zip(grads, blocks))
    gnorm = math.sqrt(sum(float(torch.sum(g * g)) for g in grads))
    gen = torch.Generator(device="cpu").manual_seed(3)
    fd_dev = []
    h = 1e-3
    for _ in range(2):
        E = [torch.randn(b.shape, generator=gen, dtype=torch.float64) for b in blocks]
        nrm = math.sqrt(sum(float(torch.sum(e * e)) for e in E))
        E = [(e / nrm).to(dev) for e in E]
        fp, _, _ = cm.cmsvd_tail_energy_grad([b.double() + h * e for b, e in zip(blocks, E)], r, ck, want_grad=False)
        fm, _, _ = cm.cmsvd_tail_energy_grad([b.double() - h * e for b, e in zip(blocks, E)], r, ck, want_grad=False)
        an = sum(float(torch.sum(g * e)) for g, e in zip(grads, E))
        fd_dev.append(abs((fp - fm) / (2 * h) - an) / gnorm)
    # exact-SVD gradient of the concatenation, for context
    Mt = torch.cat([b.double() for b in blocks], dim=1)
    lam, Uf = torch.linalg.eigh(Mt @ Mt.T)
    Ur = Uf[:, -r:]
    Gx = 2.0 * (Mt - Ur @ (Ur.T @ Mt))
    Gi = torch.cat(grads, dim=1)
    cos = float(torch.sum(Gx * Gi) / (torch.linalg.norm(Gx) * torch.linalg.norm(Gi)))
    reld = float(torch.linalg.norm(Gx - Gi) / torch.linalg.norm(Gx))
    exact_tail = float(torch.sum(lam[:-r]))
    m, k = blocks_np[0].shape
    out = {
        "metric": "tail-energy gradient steps/sec (forward + backward over the whole chain)",
        "value": round(args.steps / el, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 3),
        "forward_only_ms": round(1000.0 * fwd_s, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"shared_chain: {len(blocks)} FP32 blocks {m}x{k}, shared 96-dim subspace, "
                               f"noise 0.05, r={r}, checkpoint every {ck} steps",
                   "blocks": len(blocks), "m": int(m), "k": int(k), "r": r},
        "f": f,
        "exact_tail2": exact_tail,
        "min_cut_gap": gap,
        "euler_rel_dev": abs(euler - 2.0 * f) / (2.0 * f),
        "fd_rel_dev": fd_dev,
        "vs_exact_svd_gradient": {"cosine": cos, "rel_diff": reld},
    }
    print(json.dumps(out), flush=True)


def decision_replay(cm, h, blocks, blocks_np, clusters, r, eps, args):
    """Re-takes a seeded sample of the clustering's decisions with the oracle, in the same
    projection precision, on the device's own states: each cluster's anchor and
    acceptances are committed again in the recorded order (cmsvd_cluster_trace), an
    accepted candidate must have rel <= eps (1 + 1e-3) against the state before it, and
    a block of a later cluster rel > eps (1 - 1e-3) against the cluster's final state
    (its last pass rejected every remaining block).  Narrow candidates (<= 256 columns)
    keep the oracle's eigenvalue problems small."""
    import math

    import oracle
    from oracle import lowprec

    trace = cm.cmsvd_cluster_trace(h)
    m = int(blocks_np[0].shape[0])
    rng = np.random.default_rng(7)
    seq, off = [], 0
    for mem in clusters:
        seq.append(trace[off:off + len(mem)])
        off += len(mem)

    def ostate(st):
        S = st.S.cpu().numpy()
        keep = S > 0
        o = oracle.State(m)
        o.U = np.asfortranarray(st.U.cpu().numpy()[:, keep])
        o.sigma = S[keep].copy()
        o.energy_terms = [float(x) for x in st.acc.cpu().numpy()[:2]]
        return o

    def orel(o, j):
        e2, et = lowprec.candidate_estimate2(o, blocks_np[j], r, args.projection)
        return math.sqrt(e2 / et)

    t0 = time.perf_counter()
    acc, rej, bad = [], [], []
    later = set(range(len(blocks_np)))
    multi = [c for c, part in enumerate(seq) if len(part) > 1]
    want = set(rng.permutation(multi)[:args.replay].tolist())
    for c, part in enumerate(seq):
        later -= set(part)
        if c not in want:
            continue
        st = cm.State(m, r, blocks[0].device)
        states = []
        for j in part:
            states.append(st)
            st = cm.cmsvd_update(st, blocks[j], handle=h)
        narrow = [t for t in range(1, len(part)) if blocks_np[part[t]].shape[1] <= 256]
        for t in rng.permutation(narrow)[:1]:
            v = orel(ostate(states[t]), part[t])
            acc.append(v)
            if v > eps * (1 + 1e-3):
                bad.append(("accept", c, part[t], v))
        cand = [j for j in sorted(later) if blocks_np[j].shape[1] <= 256]
        for j in rng.permutation(cand)[:1]:
            v = orel(ostate(st), j)
            rej.append(v)
            if v <= eps * (1 - 1e-3):
                bad.append(("reject", c, j, v))
    out = {"acceptances": len(acc), "rejections": len(rej), "disagreements": len(bad),
           "max_accepted_rel": max(acc) if acc else None, "min_rejected_rel": min(rej) if rej else None,
           "seconds": round(time.perf_counter() - t0, 1)}
    log(f"decision replay {out} {bad[:3]}")
    return out


def cluster(args, cm, workloads, torch):
    """Algorithm 3 on 512 FP32 blocks with 4096 rows and widths U{64..1024} from 32
    latent 4096 x 48 subspaces (noise 1e-2), relative threshold 0.1, norm-ordered scan,
    with the candidate projections in the precision --projection selects.  Reports the
    clustering time and, on a bounded sample of narrow anchor-first pairs of the same
    collection (both widths <= 256, so that the oracle stays fast; half of them sharing a
    latent subspace), the deviation of cmsvd_merge_errors in that precision from the
    FP64 oracle; with --compare-f64 also the partition of the FP64 run."""
    r = args.rank
    t0 = time.time()
    blocks_np = workloads.latent_uneven(seed=0, nblocks=args.nblocks)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    widths = [b.shape[1] for b in blocks_np]
    log(f"generated {len(blocks)} blocks, widths {min(widths)}..{max(widths)} in {time.time() - t0:.1f}s")
    h = cm.default_handle(dev)
    h.set_projection(args.projection)
    tuned = None
    if args.autotune:
        # the scan schedule for the median candidate width, measured (or loaded) first
        ta = time.perf_counter()
        chunk = h.autotune(int(blocks_np[0].shape[0]), int(np.median(widths)), r, args.autotune)
        tuned = {"scan_chunk": chunk, "seconds": round(time.perf_counter() - ta, 3), "cache": args.autotune}
        log(f"autotuned scan chunk {tuned}")
    h.profile(True)
    h.profile_read()
    t1 = time.perf_counter()
    lab, cl, crel = cm.cmsvd_cluster(blocks, r, 0.1, sort_mode="frobenius", handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    stages = h.profile_read()
    h.profile(False)
    log(f"clustered into {len(cl)} clusters in {el:.1f}s ({args.projection} projections); stages {stages}")
    sizes = sorted((len(c) for c in cl), reverse=True)
    replay = decision_replay(cm, h, blocks, blocks_np, cl, r, 0.1, args) if args.replay > 0 else None
    versus = None
    if args.compare_f64 and args.projection != "f64":
        h.set_projection("f64")
        t2 = time.perf_counter()
        lab_f, cl_f, crel_f = cm.cmsvd_cluster(blocks, r, 0.1, sort_mode="frobenius", handle=h)
        torch.cuda.synchronize()
        versus = {"f64_seconds": round(time.perf_counter() - t2, 3), "identical_partition": lab == lab_f,
                  "f64_clusters": len(cl_f)}
        if lab == lab_f:
            versus["max_cluster_rel_diff"] = max(abs(a - b) for a, b in zip(crel, crel_f))
        log(f"FP64 run: {versus}")
        h.set_projection(args.projection)
    parity = None
    if not args.no_cpu:
        import oracle

        pairs = workloads.anchor_ordered_pairs(blocks_np)
        pairs = pairs[[widths[i] <= 256 and widths[j] <= 256 for i, j in pairs]]
        # half of the sample from pairs sharing a latent subspace (block i uses latent
        # i mod 32): those have the small relative errors where precision matters most
        same = np.array([i % 32 == j % 32 for i, j in pairs])
        rng = np.random.default_rng(2)
        n_same = min(args.parity_pairs // 2, int(same.sum()))
        cs = np.concatenate([rng.choice(np.flatnonzero(same), size=n_same, replace=False),
                             rng.choice(np.flatnonzero(~same), size=min(args.parity_pairs - n_same, int((~same).sum())),
                                        replace=False)])
        err, rel = cm.cmsvd_merge_errors(blocks, pairs[cs], r, handle=h)
        err = err.cpu().numpy()
        tc = time.perf_counter()
        e_o, rel_o = oracle.merge_errors(blocks_np, pairs[cs], r, nthreads=host_cpus()["threads"])
        ct = time.perf_counter() - tc
        dev_rel = np.abs(err - e_o) / e_o
        k = int(np.argmax(dev_rel))
        parity = {"pairs": int(len(cs)), "projection": args.projection, "max_rel_dev": float(dev_rel.max()),
                  "median_rel_dev": float(np.median(dev_rel)), "rel_at_max": float(rel_o[k]),
                  "oracle_seconds": round(ct, 1), "same_latent_pairs": int(sum(i % 32 == j % 32 for i, j in pairs[cs]))}
        log(f"parity {parity}")
    out = {
        "metric": "greedy error-constrained clustering (Algorithm 3) wall time",
        "value": round(el, 3),
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": {"f64": "f64", "bf16": "bf16 projections (fp32 accumulate), f64 core",
                  "bf16x3": "split bf16 projections (fp32 accumulate), f64 core",
                  "f32": "fp32 projections (fp32 accumulate), f64 core"}[args.projection],
        "data": "synthetic",
        "config": {"workload": f"latent_uneven: {len(blocks)} FP32 blocks 4096 x U{{64..1024}}, 32 latent 48-dim "
                               f"subspaces, noise 1e-2, r={r}, eps=0.1, frobenius order",
                   "r": r, "eps": 0.1, "projection": args.projection},
        "clusters": len(cl),
        "autotune": tuned,
        "decision_replay": replay,
        "largest_clusters": sizes[:8],
        "max_cluster_rel": max(crel) if crel else None,
        "stages_ms_launches": {k: [round(v[0], 1), v[1]] for k, v in stages.items()},
        "versus_f64": versus,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)


def cluster_residual(args, cm, workloads, torch):
    """Algorithm 2 (residual-certified clustering) on the collection of the Algorithm 3
    line: 512 FP32 blocks with 4096 rows and widths U{64..1024} from 32 latent 4096 x 48
    subspaces (noise 1e-2), relative threshold 0.1.  Reports the clustering time, the
    per-stage device time, and, on a bounded sample of narrow anchor-first pairs, the
    deviation of the chain certificate (cmsvd_residual_bound) from the FP64 oracle."""
    r = args.rank
    t0 = time.time()
    blocks_np = workloads.latent_uneven(seed=0, nblocks=args.nblocks)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    widths = [b.shape[1] for b in blocks_np]
    log(f"generated {len(blocks)} blocks, widths {min(widths)}..{max(widths)} in {time.time() - t0:.1f}s")
    h = cm.default_handle(dev)
    h.profile(True)
    h.profile_read()
    t1 = time.perf_counter()
    lab, cl, crel = cm.cmsvd_cluster_residual(blocks, r, 0.1, sort_mode=args.sort_mode, handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    stages = h.profile_read()
    h.profile(False)
    log(f"clustered into {len(cl)} clusters in {el:.2f}s; stages {stages}")
    sizes = sorted((len(c) for c in cl), reverse=True)
    parity = None
    if not args.no_cpu:
        import oracle

        n2 = [float(np.sum(b.astype(np.float64) ** 2)) for b in blocks_np]
        narrow = [i for i in range(len(blocks_np)) if widths[i] <= 128]
        rng = np.random.default_rng(3)
        picks = []
        while len(picks) < min(args.cpu_chains, len(narrow) // 2):
            i, j = (int(x) for x in rng.choice(narrow, size=2, replace=False))
            if n2[j] > n2[i]:
                i, j = j, i
            picks.append((i, j))
        worst = 0.0
        tc = time.perf_counter()
        for i, j in picks:
            b2_g, _ = cm.cmsvd_residual_bound([blocks[i], blocks[j]], r)
            b2_o, _ = oracle.residual_bound2([blocks_np[i], blocks_np[j]], r, rank_tol=-1.0)
            worst = max(worst, abs(b2_g - b2_o) / max(b2_o, 1e-12 * (n2[i] + n2[j])))
        ct = time.perf_counter() - tc
        parity = {"pairs": len(picks), "max_rel_dev_bound2": worst, "seconds": round(ct, 1),
                  "widths": [[widths[i], widths[j]] for i, j in picks]}
        log(f"parity {parity}")
    out = {
        "metric": "residual-certified clustering (Algorithm 2) wall time",
        "value": round(el, 3),
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"latent_uneven: {len(blocks)} FP32 blocks 4096 x U{{64..1024}}, 32 latent 48-dim "
                               f"subspaces, noise 1e-2, r={r}, eps=0.1, {args.sort_mode} order",
                   "r": r, "eps": 0.1},
        "clusters": len(cl),
        "largest_clusters": sizes[:8],
        "max_cluster_rel": max(crel) if crel else None,
        "stages_ms_launches": {k: [round(v[0], 1), v[1]] for k, v in stages.items()},
        "parity": parity,
    }
    print(json.dumps(out), flush=True)


def slack(args, cm, workloads, torch):
    """Estimator conservativeness (the paper's slack diagnostic): for cluster sizes
    2 .. 64 and 10 uniform block samples each, the explicit rank-r error E_r of the
    concatenation and the three estimates -- max-norm (Theorem 1), residual
    (Corollary 1) and approximate incremental (Corollary 2) -- with the blocks in the
    clustering order (largest norm first, then increasing norm).  Slack = estimate - E_r,
    both divided by ||M||_F.  Data: a 256-block pool drawn with the Table-1-like recipe
    of the chosen preset.  A few samples are re-computed by the FP64 oracle."""
    if args.preset not in SMALLK:
        raise SystemExit(f"--preset {args.preset} is a --workload table2 shape")
    nb, m, k, r = SMALLK[args.preset]
    pool = min(nb, 256)
    t0 = time.time()
    blocks_np = workloads.table1_like(seed=0, nblocks=pool, m=m, k=k)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    n2 = [float(np.sum(b.astype(np.float64) ** 2)) for b in blocks_np]
    torch.cuda.synchronize()
    log(f"generated a pool of {pool} blocks {m}x{k} in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(5)
    sizes = [2, 4, 8, 16, 32, 64]
    rows = []
    t1 = time.perf_counter()
    for size in sizes:
        for trial in range(10):
            pick = [int(i) for i in rng.choice(pool, size=size, replace=False)]
            first = max(pick, key=lambda i: (n2[i], -i))
            order = [first] + sorted((i for i in pick if i != first), key=lambda i: (n2[i], i))
            sub = [blocks[i] for i in order]
            tot = math.sqrt(sum(n2[i] for i in order))
            exact = math.sqrt(cm.cmsvd_exact_tail(sub, r))
            weyl = math.sqrt(cm.cmsvd_weyl_bound(sub, r))
            resid = math.sqrt(cm.cmsvd_residual_bound(sub, r)[0])
            st = cm.State(m, r, dev)
            for b in sub:
                st = cm.cmsvd_update(st, b, r)
            approx = float(st.est[0].item())
            rows.append({"size": size, "trial": trial, "order": order, "E": exact / tot, "max_norm": weyl / tot,
                         "residual": resid / tot, "approx": approx / tot})
        log(f"size {size} done")
    el = time.perf_counter() - t1
    summary = {}
    for size in sizes:
        sel = [x for x in rows if x["size"] == size]
        summary[str(size)] = {est: {"min": min(x[est] - x["E"] for x in sel), "median": float(np.median([x[est] - x["E"] for x in sel])),
                                    "max": max(x[est] - x["E"] for x in sel)} for est in ("max_norm", "residual", "approx")}
    parity = None
    if not args.no_cpu:
        import oracle
        from oracle import alg1, alg2

        worst = 0.0
        tc = time.perf_counter()
        checked = 0
        for x in rows:
            if x["size"] > 16 or x["trial"] != 0:
                continue
            sub = [blocks_np[i].astype(np.float64) for i in x["order"]]
            tot = math.sqrt(sum(n2[i] for i in x["order"]))
            M = np.concatenate(sub, axis=1)
            sv = np.linalg.svd(M, compute_uv=False)
            ref = {"E": math.sqrt(math.fsum((sv[r:] ** 2).tolist())) / tot,
                   "max_norm": math.sqrt(alg1.bound2(sub, r)) / tot,
                   "residual": math.sqrt(alg2.chain_bound2(sub, r)[0]) / tot,
                   "approx": float(oracle.chain_c(sub, r)[0][-1]) / tot}
            for key, v in ref.items():
                worst = max(worst, abs(x[key] - v) / max(v, 1e-6))
            checked += 1
        parity = {"samples": checked, "max_rel_dev": worst, "seconds": round(time.perf_counter() - tc, 1)}
        log(f"parity {parity}")
    neg = {est: sum(1 for x in rows if x[est] - x["E"] < -1e-9) for est in ("max_norm", "residual", "approx")}
    out = {
        "metric": "estimator slack (estimate - E_r) / ||M||_F, 10 trials per cluster size",
        "value": round(el, 3),
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"table1_like/{args.preset} pool of {pool} FP32 blocks {m}x{k}, r={r}, "
                               f"cluster sizes {sizes}, clustering order", "r": r},
        "slack": summary,
        "negative_slack_count": neg,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)


SMALLK = {  # name: (blocks, m, k, r) -- the shapes of the paper's collections
    "qualcomm": (2468, 12800, 20, 20),
    "bigearthnet": (10000, 1440, 20, 20),
    "pdebench": (5000, 3072, 67, 67),
}


# Table 2 protocol: (blocks, m, k, r, eps, noise) per collection shape of Table 1.  The
# values are synthetic (64 latent 16-dim subspaces plus Gaussian noise); the noise puts
# the per-block noise-to-signal energy at 1e-3 (1e-2 for the 20 % SmolVLM threshold), so
# that clusters of one latent subspace fit the error threshold.
TABLE2 = {
    "qualcomm": (2468, 12800, 20, 20, 0.05, 1.12e-3),
    "bigearthnet": (10000, 1440, 20, 20, 0.05, 3.33e-3),
    "pdebench": (5000, 3072, 67, 67, 0.05, 2.28e-3),
    "smolvlm": (333760, 768, 1, 32, 0.20, 1.44e-2),
}


def table2(args, cm, workloads, torch):
    """The paper's Table 2 protocol on a synthetic collection of one Table 1 shape: the
    five clustering variants (max norm = Algorithm 1; residual = Algorithm 2 with norm or
    residual sorting; approximate = Algorithm 3 with norm or residual sorting) at the
    shape's rank and threshold, each followed by the compression back-end.  Reports per
    variant the clustering wall time (decomposition excluded, as in the paper), the time
    relative to max norm, the compression ratio, the realised relative error and the
    number of clusters.  --pool takes the first N blocks of the collection (the SmolVLM
    shape defaults to 20,000 of its 333,760 one-column blocks)."""
    nb, m, k, r, eps, noise = TABLE2[args.preset]
    pool = args.pool if args.pool > 0 else (20000 if args.preset == "smolvlm" else nb)
    pool = min(pool, nb)
    t0 = time.time()
    blocks_np = workloads.table1_like(seed=0, nblocks=pool, m=m, k=k, noise=noise)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    log(f"generated {pool} blocks {m}x{k} in {time.time() - t0:.1f}s")
    h = cm.default_handle(dev)
    variants = [
        ("max norm", lambda: cm.cmsvd_cluster_weyl(blocks, r, eps, handle=h)),
        ("res. (norm sorting)", lambda: cm.cmsvd_cluster_residual(blocks, r, eps, "frobenius", handle=h)),
        ("res. (res. sorting)", lambda: cm.cmsvd_cluster_residual(blocks, r, eps, "residual", handle=h)),
        ("approx. (norm sorting)", lambda: cm.cmsvd_cluster(blocks, r, eps, "frobenius", handle=h)),
        ("approx. (res. sorting)", lambda: cm.cmsvd_cluster(blocks, r, eps, "residual", handle=h)),
    ]
    rows = []
    for name, run in variants:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lab, cl, crel = run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        t2 = time.perf_counter()
        _, summ = cm.compress_partition(blocks, lab, r, handle=h)
        torch.cuda.synchronize()
        ct = time.perf_counter() - t2
        sizes = sorted((len(c) for c in cl), reverse=True)
        row = {"method": name, "seconds": round(el, 3), "compression_ratio": round(summ["compression_ratio"], 4),
               "rel_error": round(summ["rel_error"], 5), "clusters": len(cl), "largest": sizes[:4],
               "max_cluster_rel": round(max(crel), 5) if crel else None, "compress_seconds": round(ct, 2)}
        rows.append(row)
        log(f"{name}: {row}")
    base = rows[0]["seconds"]
    for row in rows:
        row["relative_time"] = round(row["seconds"] / base, 2) if base > 0 else None
    out = {
        "metric": "Table 2 protocol: compression ratio and clustering wall time per variant",
        "unit": "s",
        "n_gpus": 1,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"table1_like/{args.preset}: {pool} of {nb} FP32 blocks {m}x{k}, 64 latent 16-dim "
                               f"subspaces, noise {noise}, r={r}, eps={eps}",
                   "blocks": pool, "m": m, "k": k, "r": r, "eps": eps},
        "variants": rows,
        "all_within_eps": all(row["rel_error"] <= eps + 1e-9 for row in rows),
    }
    print(json.dumps(out), flush=True)


def smallk_vectors(args, cm, workloads, torch):
    """The one-column SmolVLM shape at full size: 333,760 candidate blocks of 768 x 1 and
    r = 32.  A pair of single vectors has rank 2 <= r (an exact zero error), so the unit
    measured is Algorithm 3's scan step once a cluster holds more than r vectors: every
    candidate against 64 cluster matrices of 64 vectors each (one per latent subspace,
    768 x 64, truncated to rank 32 inside the call), 21,360,640 merges in one
    cmsvd_merge_errors call per step.  Values from the Table 2 recipe (64 latent 16-dim
    subspaces, noise-to-signal energy 1e-2); the candidates live in one device matrix and
    are passed as column views.  Sampled parity against the FP64 oracle."""
    nb, m, r, na, per = 333760, 768, 32, 64, 64
    noise = TABLE2["smolvlm"][5]
    t0 = time.time()
    vecs = workloads.table1_like(seed=0, nblocks=na * per + nb, m=m, k=1, noise=noise)
    anchors_np = [np.hstack([vecs[g + na * i] for i in range(per)]) for g in range(na)]
    cand_np = np.hstack(vecs[na * per:])
    del vecs
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    anchors = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in anchors_np]
    cand = torch.from_numpy(np.ascontiguousarray(cand_np)).to(dev)
    blocks = cm.BlockArray(anchors + [cand[:, j:j + 1] for j in range(nb)])  # marshalled once
    pairs = np.empty((na * nb, 2), dtype=np.int32)
    pairs[:, 0] = np.repeat(np.arange(na, dtype=np.int32), nb)
    pairs[:, 1] = np.tile(np.arange(na, na + nb, dtype=np.int32), na)
    torch.cuda.synchronize()
    log(f"generated {na} cluster matrices {m}x{per} and {nb} candidates {m}x1 in {time.time() - t0:.1f}s")
    h = cm.Handle(dev)
    for w in range(args.warmup):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup}")
    h.profile(True)
    h.profile_read()
    t1 = time.perf_counter()
    for st in range(args.steps):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
        torch.cuda.synchronize()
        log(f"step {st + 1}/{args.steps}")
    el = time.perf_counter() - t1
    stages = h.profile_read()
    h.profile(False)
    err_h = err.cpu().numpy()
    rel_h = rel.cpu().numpy()
    parity = None
    if not args.no_cpu:
        import oracle

        rng = np.random.default_rng(4)
        cs = rng.choice(len(pairs), size=min(args.cpu_pairs, len(pairs)), replace=False)
        sub = [anchors_np[a] for a in range(na)] + [cand_np[:, j - na:j - na + 1] for j in pairs[cs, 1]]
        sp = np.stack([pairs[cs, 0], na + np.arange(len(cs))], axis=1).astype(np.int32)
        e_o, _ = oracle.merge_errors(sub, sp, r, nthreads=host_cpus()["threads"])
        dev_rel = np.abs(err_h[cs] - e_o) / e_o
        parity = {"pairs": int(len(cs)), "max_rel_dev": float(dev_rel.max())}
        log(f"parity {parity}")
    out = {
        "metric": "candidate merges evaluated/sec (every candidate against every cluster matrix, one call per step)",
        "value": round(len(pairs) * args.steps / el, 2),
        "unit": "merges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 3),
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"table1_like/smolvlm: {nb} FP32 candidates {m}x1 against {na} cluster matrices "
                               f"{m}x{per}, 64 latent 16-dim subspaces, noise {noise:.3g}, r={r}",
                   "candidates": nb, "clusters": na, "m": m, "k": 1, "r": r, "pairs": int(len(pairs))},
        "stages_ms_per_step": {n: round(stages[n][0] / args.steps, 3) for n in stages},
        "parity": parity,
        "mean_rel": float(np.mean(rel_h)),
    }
    print(json.dumps(out), flush=True)


def smallk(args, cm, workloads, torch):
    """All anchor-first pairs of a collection with the paper's shapes (Table 1: many thin
    blocks) and synthetic values (64 latent 16-dim subspaces + noise 0.05), evaluated in
    one cmsvd_merge_errors call per step; sampled parity against the FP64 oracle.  The
    one-column SmolVLM shape runs smallk_vectors instead."""
    if args.preset == "smolvlm":
        return smallk_vectors(args, cm, workloads, torch)
    if args.preset not in SMALLK:
        raise SystemExit(f"--preset {args.preset} is a --workload table2 shape")
    nb, m, k, r = SMALLK[args.preset]
    t0 = time.time()
    blocks_np = workloads.table1_like(seed=0, nblocks=nb, m=m, k=k)
    pairs = workloads.anchor_ordered_pairs(blocks_np)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(b).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    log(f"generated {nb} blocks {m}x{k} and {len(pairs)} pairs in {time.time() - t0:.1f}s")
    h = cm.Handle(dev)
    for w in range(args.warmup):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup}")
    h.profile(True)
    h.profile_read()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    stages = h.profile_read()
    h.profile(False)
    err_h = err.cpu().numpy()
    parity = None
    if not args.no_cpu:
        import oracle

        rng = np.random.default_rng(4)
        cs = rng.choice(len(pairs), size=min(args.cpu_pairs, len(pairs)), replace=False)
        e_o, _ = oracle.merge_errors(blocks_np, pairs[cs], r, nthreads=host_cpus()["threads"])
        nrm = np.array([math.sqrt(float(np.sum(blocks_np[i].astype(np.float64) ** 2)) +
                                  float(np.sum(blocks_np[j].astype(np.float64) ** 2))) for i, j in pairs[cs]])
        dev_rel = np.abs(err_h[cs] - e_o) / np.maximum(e_o, 1e-6 * nrm)
        parity = {"pairs": int(len(cs)), "max_rel_dev": float(dev_rel.max())}
        log(f"parity {parity}")
    out = {
        "metric": "candidate merges evaluated/sec (all anchor-first pairs, one call per step)",
        "value": round(len(pairs) * args.steps / el, 2),
        "unit": "merges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 3),
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"table1_like/{args.preset}: {nb} FP32 blocks {m}x{k}, 64 latent 16-dim "
                               f"subspaces, noise 0.05, r={r}, all {len(pairs)} anchor-first pairs",
                   "blocks": nb, "m": m, "k": k, "r": r, "pairs": int(len(pairs))},
        "stages_ms_per_step": {n: round(stages[n][0] / args.steps, 3) for n in stages},
        "parity": parity,
        "mean_rel": float(np.mean(rel.cpu().numpy())),
    }
    print(json.dumps(out), flush=True)


def weights(args, cm, workloads, torch):
    """224 FP32 weight-shaped blocks of 4096 x 4096 (32 layers x 7 projections) in 8
    chains of 28; each block is appended as 8 panels of 512 columns and the 8 chains
    advance together (one cmsvd_update_batch per panel step, 224 steps), r = 512.
    Checks that hold at any size: the plug-in error equals the discarded-energy tally,
    and the estimate is non-decreasing along every chain and below ||M||_F."""
    r, npan = 512, 8
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    blocks = workloads.weight_like_torch(seed=0, device=dev)
    torch.cuda.synchronize()
    log(f"generated {len(blocks)} blocks {tuple(blocks[0].shape)} on the device in {time.time() - t0:.1f}s")
    chains = [blocks[28 * g:28 * (g + 1)] for g in range(8)]
    w = blocks[0].shape[1] // npan
    m = blocks[0].shape[0]
    h = cm.Handle(dev)
    states = [cm.State(m, r, dev) for _ in range(8)]
    hist = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for step in range(28 * npan):
        b, p = divmod(step, npan)
        states = cm.cmsvd_update_batch(states, [ch[b][:, w * p:w * (p + 1)] for ch in chains], r, handle=h)
        if p == npan - 1:
            torch.cuda.synchronize()
            hist.append(torch.stack([s.est for s in states]).cpu().numpy())
            log(f"block {b + 1}/28 of every chain done, {time.perf_counter() - t1:.1f}s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    hist = np.array(hist)  # (28, 8, 2)
    etot = np.array([[float(s.acc[0] + s.acc[1]) for s in states]])
    out = {
        "metric": "incremental rank-512 estimate over 8 chains of 28 weight-shaped blocks (8 panels each)",
        "value": round(el, 3),
        "unit": "s",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "weight_like: 224 FP32 blocks 4096x4096 (sigma_i = i^-0.8, 8 shared 512-dim bases, "
                               "30% fresh directions), 8 chains x 28 blocks x 8 panels of 512, r=512",
                   "chains": 8, "blocks_per_chain": 28, "panels": npan, "r": r},
        "ms_per_panel_step": round(1000.0 * el / (28 * npan), 3),
        "final_rel": (hist[-1, :, 0] / np.sqrt(etot[0])).tolist(),
        "plugin_vs_discarded_max_rel": float(np.max(np.abs(hist[..., 0] ** 2 - hist[..., 1] ** 2)
                                               / np.maximum(hist[..., 0] ** 2, 1e-300))),
        "monotone": bool(np.all(np.diff(hist[..., 0], axis=0) >= -1e-12 * hist[1:, :, 0])),
        "below_norm": bool(np.all(hist[-1, :, 0] <= np.sqrt(etot[0]))),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-pairs", type=int, default=48, help="0 skips the plain per-pair leg")
    ap.add_argument("--library-pairs", type=int, default=16,
                    help="pairs of the library-form context leg (torch FP64 SVDs); 0 skips it")
    ap.add_argument("--cpu-pairs", type=int, default=448, help="oracle sample size (about 17 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--groups", type=int, default=16)
    ap.add_argument("--per-group", type=int, default=16)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of MIB MiB (FP64) three times, the reference "
                         "dispatch for scaling the HBM traffic counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, "
                         "WRITE_SIZE) of a run with --calibrate-copy, then exit")
    ap.add_argument("--pmc-mib", type=int, default=1024, help="copy size used with --pmc-summary")
    ap.add_argument("--no-check", action="store_true", help="chain_grad: skip the finite-difference and "
                    "exact-SVD checks (for profiling)")
    ap.add_argument("--rank", type=int, default=32, help="cluster: target rank (32 or 128)")
    ap.add_argument("--nblocks", type=int, default=512, help="cluster: collection size")
    ap.add_argument("--pool", type=int, default=0, help="table2: blocks used (0: the preset's default)")
    ap.add_argument("--preset", default="qualcomm", choices=("qualcomm", "bigearthnet", "pdebench", "smolvlm"),
                    help="smallk, slack, table2: collection shape (Table 1 of the paper; values synthetic)")
    ap.add_argument("--sort-mode", default="frobenius", choices=("frobenius", "residual"),
                    help="cluster_residual: candidate order of a pass")
    ap.add_argument("--cpu-chains", type=int, default=6, help="cluster_residual: oracle sample (narrow pairs)")
    ap.add_argument("--graph-steps", type=int, default=5,
                    help="pairs: steps replayed from a captured HIP graph after the timed eager steps (0: none)")
    ap.add_argument("--autotune", default=None, metavar="CACHE",
                    help="cluster: tune the scan schedule first (JSON cache path; loaded when present)")
    ap.add_argument("--replay", type=int, default=0,
                    help="cluster: clusters whose decisions the oracle re-takes on the device states")
    ap.add_argument("--projection", default="f32", choices=("f64", "bf16", "bf16x3", "f32"),
                    help="pairs, cluster: precision of the candidate projections")
    ap.add_argument("--compare-f64", action="store_true", help="cluster: also run the FP64 clustering")
    ap.add_argument("--parity-pairs", type=int, default=48, help="cluster: oracle sample (narrow pairs)")
    ap.add_argument("--workload", default="pairs",
                    choices=("pairs", "chain_grad", "cluster", "cluster_residual", "smallk", "weights", "slack",
                             "table2"),
                    help="pairs: batched merge errors (the default line); chain_grad: tail energy and "
                         "its gradient along a 64-block chain")
    args = ap.parse_args()
    if args.pmc_summary:
        nb = args.groups * args.per_group
        rec = pmc_summary(*args.pmc_summary, copy_mib=args.pmc_mib)
        rec["pairs"] = nb * (nb - 1) // 2
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the pair "
              "list across GPUs is described in the design notes but not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy > 0:
        # reference dispatches for the traffic counters: dst = 1.0 * src reads and writes
        # exactly MIB MiB each; the kernel name carries "MulFunctor"
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: 3 dispatches of {nbytes} bytes read + written")

    import paper_2601_11626_amd as cm
    import workloads

    if args.workload == "chain_grad":
        return chain_grad(args, cm, workloads, torch)
    if args.workload == "cluster":
        return cluster(args, cm, workloads, torch)
    if args.workload == "cluster_residual":
        return cluster_residual(args, cm, workloads, torch)
    if args.workload == "smallk":
        return smallk(args, cm, workloads, torch)
    if args.workload == "table2":
        return table2(args, cm, workloads, torch)
    if args.workload == "slack":
        return slack(args, cm, workloads, torch)
    if args.workload == "weights":
        return weights(args, cm, workloads, torch)

    r = 64
    t0 = time.time()
    blocks_np = workloads.rotated_groups(seed=0, groups=args.groups, per_group=args.per_group)
    pairs = workloads.anchor_ordered_pairs(blocks_np)
    log(f"generated {len(blocks_np)} blocks {blocks_np[0].shape} and {len(pairs)} pairs in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    blocks = [torch.from_numpy(np.ascontiguousarray(b)).to(dev) for b in blocks_np]
    torch.cuda.synchronize()
    h = cm.Handle(dev)
    h.set_projection(args.projection)
    m, k = blocks_np[0].shape
    npairs = len(pairs)

    # warmup (also grows the workspace)
    for w in range(args.warmup):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    h.profile(True)
    h.profile_read()  # reset
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.steps):
        err, rel = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    stages = h.profile_read()
    h.profile(False)
    log(f"timed {args.steps} steps in {elapsed:.3f}s; stages {stages}")
    value = npairs * args.steps / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps
    err_h = err.cpu().numpy()
    rel_h = rel.cpu().numpy()

    # The same step replayed from a captured HIP graph (cmsvd_options.graphs): the first
    # call runs eagerly, the second is captured (its wall time reported apart), and the
    # timed replays launch the graph on the same stream.
    graph = None
    if args.graph_steps > 0:
        hg = cm.Handle(dev, projection=args.projection, graphs=True)
        out = (torch.empty(npairs, dtype=torch.float64, device=dev), torch.empty(npairs, dtype=torch.float64, device=dev))
        barr = cm.BlockArray(blocks)
        for _ in range(2):
            cm.cmsvd_merge_errors(barr, pairs, r, handle=hg, out=out)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.graph_steps):
            cm.cmsvd_merge_errors(barr, pairs, r, handle=hg, out=out)
        torch.cuda.synchronize()
        gel = time.perf_counter() - tg
        gs = hg.graph_stats()
        gdev = float(np.max(np.abs(out[0].cpu().numpy() - err_h) / np.maximum(err_h, 1e-300)))
        graph = {"value": round(npairs * args.graph_steps / gel, 2), "unit": "merges/s", "steps": args.graph_steps,
                 "ms_per_step": round(1000.0 * gel / args.graph_steps, 3), "capture_ms": round(gs["last_capture_ms"], 3),
                 "captures": gs["captures"], "replays": gs["replays"], "max_rel_diff_vs_eager": gdev}
        log(f"graph replays: {graph}")
        hg.close()

    # plain per-pair method on a sample of the same pairs
    rng = np.random.default_rng(1)
    plain = None
    if args.plain_pairs > 0:
        sample = rng.choice(npairs, size=min(args.plain_pairs, npairs), replace=False)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        plain_err = []
        for p in sample:
            e, _ = cm.cmsvd_merge_errors(blocks, pairs[p:p + 1], r, handle=h)
            plain_err.append(e)
        torch.cuda.synchronize()
        plain_rate = len(sample) / (time.perf_counter() - tp)
        plain_err = torch.cat(plain_err).cpu().numpy()
        plain_dev = float(np.max(np.abs(plain_err - err_h[sample]) / np.maximum(err_h[sample], 1e-300)))
        plain = {"value": round(plain_rate, 3), "unit": "merges/s", "pairs": int(len(sample)),
                 "max_rel_diff_vs_batched": plain_dev}
        log(f"plain: {plain_rate:.1f} merges/s over {len(sample)} pairs")

    # The same per-pair math in library form, for context: the anchor's truncation from
    # torch's FP64 SVD, then the singular values of [U_r S_r, A_j] (rocSOLVER/rocBLAS).
    library = None
    if args.library_pairs > 0:
        sample = rng.choice(npairs, size=min(args.library_pairs, npairs), replace=False)
        torch.cuda.synchronize()
        tl = time.perf_counter()
        lib_err = []
        for p in sample:
            i, j = int(pairs[p, 0]), int(pairs[p, 1])
            A = blocks[i].double()
            B = blocks[j].double()
            U, S, _ = torch.linalg.svd(A, full_matrices=False)
            sv = torch.linalg.svdvals(torch.cat([U[:, :r] * S[:r], B], dim=1))
            e2 = torch.sum(S * S) + torch.sum(B * B) - torch.sum(sv[:r] ** 2)
            lib_err.append(torch.sqrt(torch.clamp(e2, min=0.0)))
        lib_err = torch.stack(lib_err).cpu().numpy()
        lib_rate = len(sample) / (time.perf_counter() - tl)
        lib_dev = float(np.max(np.abs(lib_err - err_h[sample]) / np.maximum(err_h[sample], 1e-300)))
        library = {"value": round(lib_rate, 3), "unit": "merges/s", "pairs": int(len(sample)),
                   "kind": "torch FP64 per pair: svd of the anchor, svdvals of [U_r S_r, A_j]",
                   "max_rel_diff_vs_batched": lib_dev}
        log(f"library: {lib_rate:.1f} merges/s over {len(sample)} pairs")

    # dominant stage and its roofline position.  Cores of order 193..320 are
    # tridiagonalised for n - 192 column steps by EIG_KERNEL; the trailing 192 x 192
    # matrix goes to the TAIL_KERNELS (stage core_tail).  Each stage is priced at the
    # (4/3) n^3 of the part of the reduction it does.
    n_core = r + k
    nt = TAIL_ORDER if TAIL_ORDER < n_core <= 320 else 0
    flops = {
        "projection": 2.0 * r * k * m * npairs * args.steps,
        "core_eig": (4.0 / 3.0) * (float(n_core) ** 3 - float(nt) ** 3) * npairs * args.steps,
        "core_tail": (4.0 / 3.0) * float(nt) ** 3 * npairs * args.steps,
    }
    timed = {n: stages[n][0] for n in ("commit", "projection", "core_eig", "core_bisect", "core_tail")}
    dom = max(timed, key=timed.get)
    roof = None
    if dom in flops and timed[dom] > 0 and not (dom == "projection" and args.projection != "f64"):
        ach = flops[dom] / (timed[dom] * 1e-3) / 1e12
        label = {"core_eig": EIG_KERNEL + (f" (tridiagonalisation, first n - {nt} steps)" if nt else
                                           " (tridiagonalisation)"),
                 "core_tail": f"trailing {nt} x {nt}: " + " + ".join(TAIL_KERNELS),
                 "projection": "gemm_f64_kernel (Y = U^T B)"}[dom]
        roof = {
            "kernel": label,
            "bound": "mfma" if dom == "projection" else "alu",
            "achieved": round(ach, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP64_TFLOPS, 4),
            "traffic": None,
            "launches": int(stages[dom][1]),
            "avg_launch_ms": round(timed[dom] / max(stages[dom][1], 1), 3),
        }
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": None, "traffic": None}

    if roof.get("achieved") is not None and dom in ("core_eig", "projection"):
        roof["traffic"] = measured_traffic(EIG_KERNEL if dom == "core_eig" else "gemm_f64_kernel", npairs)

    # the trailing tridiagonalisation against the same FP64 vector peak
    tail_roof = None
    if timed["core_tail"] > 0:
        ach = flops["core_tail"] / (timed["core_tail"] * 1e-3) / 1e12
        tail_roof = {"kernel": f"trailing {nt} x {nt}: " + " + ".join(TAIL_KERNELS),
                     "bound": "alu", "achieved": round(ach, 3),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                     "launches": int(stages["core_tail"][1]),
                     "avg_launch_ms": round(timed["core_tail"] / max(stages["core_tail"][1], 1), 3)}

    # the projection GEMMs against the matrix-core peak of their own operand type
    proj_roof = None
    if timed["projection"] > 0:
        pk, kern = PROJ_PEAK[args.projection]
        ach = flops["projection"] / (timed["projection"] * 1e-3) / 1e12
        proj_roof = {"kernel": kern, "bound": "mfma", "achieved": round(ach, 3), "peak": pk, "unit": "TFLOP/s",
                     "frac": round(ach / pk, 4), "launches": int(stages["projection"][1]),
                     "avg_launch_ms": round(timed["projection"] / max(stages["projection"][1], 1), 3)}

    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle

        hc = host_cpus()
        nthreads = hc["threads"]
        cs = rng.choice(npairs, size=min(args.cpu_pairs, npairs), replace=False)
        tc = time.perf_counter()
        e_o, rel_o = oracle.merge_errors(blocks_np, pairs[cs], r, nthreads=nthreads)
        ct = time.perf_counter() - tc
        cpu = {
            "value": round(len(cs) / ct, 4),
            "unit": "merges/s",
            "cores": nthreads,
            "host": hc,
            "kind": "oracle",
            "sample": f"{len(cs)} random anchor-first pairs of the same 256-block collection "
                      f"(each with its own anchor truncation), {ct:.1f}s wall",
        }
        nrm = np.array([math.sqrt(float(np.sum(blocks_np[i].astype(np.float64) ** 2)) +
                                  float(np.sum(blocks_np[j].astype(np.float64) ** 2))) for i, j in pairs[cs]])
        g = err_h[cs]
        dev_rel = np.abs(g - e_o) / np.maximum(e_o, 1e-6 * nrm)
        parity = {"pairs": int(len(cs)), "max_rel_dev": float(dev_rel.max()),
                  "max_sq_dev_over_norm2": float(np.max(np.abs(g ** 2 - e_o ** 2) / nrm ** 2))}
        log(f"cpu oracle: {cpu}; parity {parity}")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "merges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.projection == "f64" else f"f64 core, {args.projection} projections",
        "data": "synthetic",
        "config": {
            "projection": args.projection,
            "workload": f"rotated_groups: {len(blocks_np)} FP32 blocks {m}x{k}, r={r}, all {npairs} anchor-first "
                        f"pairs per step (anchor init included)",
            "blocks": len(blocks_np), "m": int(m), "k": int(k), "r": r, "pairs": npairs,
        },
        "plain": plain,
        "speedup_vs_plain": round(value / plain["value"], 2) if plain else None,
        "graph": graph,
        "library": library,
        "stages_ms_per_step": {n: round(stages[n][0] / args.steps, 3) for n in stages},
        "roofline": roof,
        "tail_roofline": tail_roof,
        "projection_roofline": proj_roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "mean_rel": float(np.mean(rel_h)),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the FastPI hot path on one MI355X.

One step = the whole device path on resident inputs: value split (a1), block SVDs (a2),
row update (a3), column update (a4), unpermute (a5) and the pseudoinverse apply
Z = V Sigma^+ U^T Y (a6), for the workload 100000 x 5000 (0.2% dense, power-law 1.9,
lognormal values, 1000 Bernoulli(0.005) labels, alpha 0.1) unless --config says otherwise.
The host reordering and planning run once before the timed region (their time is
reported separately as plan_s).

Prints one JSON line. `value` is the algorithmic throughput F_model / T_step in TFLOP/s,
where F_model is the flop count of the method's Brand-form update terms (see flop_model()).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import scipy.sparse as sp  # noqa: E402


def progress(msg):
    """Progress lines on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def svd_thin_flops(p, q):
    """Golub & Van Loan R-SVD count for a thin SVD of a p x q matrix with both factors:
    6 P Q^2 + 20 Q^3 with P = max(p, q), Q = min(p, q)."""
    p, q = max(p, q), min(p, q)
    if q <= 0:
        return 0.0
    return 6.0 * p * q * q + 20.0 * q ** 3


def qr_thin_flops(p, q):
    """Householder QR of a p x q matrix with k = min(p, q) reflectors (R: 4pqk - 2(p+q)k^2
    + 4k^3/3, i.e. 2pq^2 - 2q^3/3 when p >= q), doubled for the thin Q."""
    k = min(p, q)
    if k <= 0:
        return 0.0
    return 2.0 * (4.0 * p * q * k - 2.0 * (p + q) * k * k + 4.0 * k ** 3 / 3.0)


def border_counts(plan, indptr, indices):
    """nnz(A21), nnz(T) and the sum over A21's entries of the rank of the diagonal block its
    column belongs to (the cost of P2 = V1^T A21^T), from the host CSR and the plan's
    permutation and block table."""
    i = plan.info
    piT, piF = plan.permutation()
    rows = np.repeat(np.arange(i["m"]), np.diff(indptr))
    r_new = piT[rows]
    c_new = piF[np.asarray(indices)]
    in_t = c_new >= i["n1"]
    in_a21 = (r_new >= i["m1"]) & ~in_t
    blocks, ranks = plan.blocks(), plan.block_ranks()
    col_rank = np.zeros(max(i["n1"], 1), dtype=np.int64)
    for (_, c0, _, ni), s in zip(blocks, ranks):
        col_rank[c0:c0 + ni] = s
    return int(in_a21.sum()), int(in_t.sum()), float(col_rank[c_new[in_a21]].sum())


def flop_model(plan, blocks, ranks, L, indptr, indices):
    """Algorithmic flops of one step (precision-independent), the Brand-form terms of the
    incremental updates. rho2 = min(n1 - s_b, m2) and rho3 = min(m - s, n2) are the generic
    ranks of the two residuals (each lies in the complement of s_b or s directions).
    a2: a thin SVD of every dense diagonal block (Eq. 1);
    a3 (Eq. 2): P2 = V1^T A21^T, R2 = A21^T - V1 P2, the thin QR of R2, the core SVD of
        (s_b + rho2) x (s_b + m2), U1 Ut_top and V2 = [V1 Q2] Uhat;
    a4 (Eq. 3): P3 = U2^T T and R3 = T - U2 P3 twice (a second Gram-Schmidt pass), the thin QR
        of R3, the core SVD of (s + rho3) x (s + n2), U = [U2 Q3] Uhat and V2 Vt_top;
    a6: U^T Y, Sigma^+ W and V W."""
    i = plan.info
    m, n, m2, n1, n2 = i["m"], i["n"], i["m2"], i["n1"], i["n2"]
    s_b, s, r = i["s_b"], i["s"], i["r"]
    nnz21, nnzT, p2_terms = border_counts(plan, indptr, indices)
    f2 = sum(svd_thin_flops(bm, bn) for (_, _, bm, bn) in blocks if bm > 0 and bn > 0)
    sum_ms = float(sum(int(bm) * int(sv) for (_, _, bm, _), sv in zip(blocks, ranks)))
    sum_ns = float(sum(int(bn) * int(sv) for (_, _, _, bn), sv in zip(blocks, ranks)))
    rho2 = max(0, min(n1 - s_b, m2))
    rho3 = max(0, min(m - s, n2))
    f3 = 0.0
    if n1 > 0:
        f3 = (2.0 * p2_terms + 2.0 * sum_ns * m2 + qr_thin_flops(n1, m2)
              + svd_thin_flops(s_b + m2, s_b + rho2) + 2.0 * sum_ms * s + 2.0 * n1 * (s_b + rho2) * s)
    f4 = (2.0 * (2.0 * nnzT * s + 2.0 * m * s * n2) + qr_thin_flops(m, n2)
          + svd_thin_flops(s + n2, s + rho3) + 2.0 * m * (s + rho3) * r + 2.0 * n1 * s * r)
    f6 = 2.0 * m * r * L + r * L + 2.0 * n * r * L
    return {"a2": f2, "a3": f3, "a4": f4, "a6": f6, "total": f2 + f3 + f4 + f6,
            "rho2": rho2, "rho3": rho3, "nnz_A21": nnz21, "nnz_T": nnzT}


# Per-unit algorithmic work of the eigensolver's pair solve (k_eig_solve): one cyclic Jacobi
# sweep of a 32 x 32 symmetric pair matrix = 31 steps, each updating all 1024 entries of H
# (4 multiplies + 3 adds) and of W (2 multiplies + 1 add): 31 * 1024 * 10 flops; the
# partial-Gram sum adds nchunk * 1024 flops.
PAIR_SWEEP_FLOPS = 31 * 1024 * 10
GRAM_ROWS = 128          # default rows per partial Gram (eigensolver)
BW = 16                  # eigensolver column block


# HBM bytes per launch of a timed kernel, from the two counter runs summarised under
# profiles/ (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the scales read off a 256 MiB device copy in
# the same runs), keyed by (kernel, workload, precision of the timed form), with the digest
# of the kernel source they were taken on and the core-solver settings of that run (they set
# the basis sizes, hence the bytes of a launch); the eigensolver kernels' figures are per
# partial-Gram height (rows per chunk: it sets how many partials a pair solve reads). The
# figure is dropped (null) for any other workload, as soon as the kernel's source differs,
# and for other core-solver settings or chunk heights.
TRAFFIC_CORE = {"mode": 1, "min_order": 1024, "k_factor": 2.0, "k_factor_mixed": 1.5, "max_frac": 0.65,
                "iters_fp64": 28, "iters_mixed": 18, "orth_every": 2}
TRAFFIC = {
    ("cq_panel", "c3", "mixed"): (1503334, "subspace.hip", "__device__ int cq_factor_invert(", "// After panel p:",
                                  "034fe9c71c7400a65c362deb844ee215d67250e14fe77a159f508a1b9b223686"),
    ("eig_solve", "c3", "mixed"): ({128: 1027891, 64: 1807053}, "eig.hip", "__device__ __forceinline__ void pair_solve(",
                                   "// X[:, I u J] <- X[:, I u J] W over a tile",
                                   "c2f5ba0ce77ef0efbbd63cf84a9049359fb102d74557ba2d6f2ea1dfaf8a4f72"),
    ("eig_round", "c3", "mixed"): ({128: 10183885, 64: 9873818}, "eig.hip",
                                   "template <int ROWS>\n__global__ __launch_bounds__(256) void k_eig_round(",
                                   "// End of a sweep:",
                                   "4a92ac0365fbc8a47656ae36c9ce1a75a33b9b20be34470f03ccecc02601554b"),
    # the products by G: the kernel and the K-split rule of the subspace route (the row-map
    # template flag added since the counter runs leaves this instantiation's machine code
    # unchanged but for one kernel-argument offset)
    ("sub_gemm", "c3", "mixed"): (280014746, ("mfma_gemm.hip", "driver.cpp"),
                                  ("template <typename Tc, bool TA, bool TB, bool GA>",
                                   "// the q x k products by G (128 x 128 tiles)"),
                                  ("// C (M x N, ldc) = op(A) op(B)", "const int64_t kp = R.kp;"),
                                  "e9fceb3404bfb4d826f0c0c792c5ece00074200f0b63e9f389827c8f0cff628a"),
}


def kernel_traffic(kname, config, precision, core=None, tuning=None):
    key = (kname, config, precision)
    if key not in TRAFFIC:
        return None
    if core is not None and any(abs(float(core.get(f, -1)) - float(v)) > 1e-12 for f, v in TRAFFIC_CORE.items()):
        return None
    import hashlib
    nbytes, fname, start, end, digest = TRAFFIC[key]
    if nbytes is None:
        return None
    if isinstance(nbytes, dict):
        rows = (tuning or {}).get("gram_rows", GRAM_ROWS)
        if rows not in nbytes:
            return None
        nbytes = nbytes[rows]
    # one source section, or several (kernel and launch rule) hashed in order
    sections = [(fname, start, end)] if isinstance(fname, str) else list(zip(fname, start, end))
    text = ""
    for fn, st, en in sections:
        with open(os.path.join(ROOT, "paper_2011_04235_amd", "csrc", fn)) as f:
            src = f.read()
        a = src.index(st)
        b = src.index(en, a + 1) if en else len(src)
        text += src[a:b]
    if hashlib.sha256(text.encode()).hexdigest() != digest:
        return None
    return nbytes


# HBM bytes per call of the label SpMM (k_label_spmm + k_label_reduce) on the 300000 x 10000
# labelled workload from the counter runs summarised in profiles/label_spmm_c5_pmc.md, with the
# digest of the kernel source they were taken on (null for other workloads or another source).
LABEL_SPMM_TRAFFIC_BYTES = {"c5": 1230828237}
LABEL_SPMM_DIGEST = "a3b3a0e0565694f0ea9b3e92443b5a19ef557d51d928d384045c64e120312663"


def label_spmm_traffic(config):
    if config not in LABEL_SPMM_TRAFFIC_BYTES:
        return None
    import hashlib
    with open(os.path.join(ROOT, "paper_2011_04235_amd", "csrc", "evaluate.hip")) as f:
        src = f.read()
    a = src.index("// Label SpMM of the sparse-label apply")
    b = src.index("int label_spmm_chunks(", a)
    if hashlib.sha256(src[a:b].encode()).hexdigest() != LABEL_SPMM_DIGEST:
        return None
    return LABEL_SPMM_TRAFFIC_BYTES[config]


def eig_shape(q, gram_rows=128):
    ld = (q + BW - 1) // BW * BW
    nblk = ld // BW
    nbe = nblk + (nblk & 1)
    return ld, nblk, nbe // 2, nbe - 1, (ld + gram_rows - 1) // gram_rows


def eig_job_flops(order, sw, rot, tuning, kernel):
    """Algorithmic flops of one eigensolve's launches of `kernel` over a run of `sw` sweeps
    in which `rot` pair solves ran (the others found their pair orthogonal already).
    k_eig_solve: every pair solve that ran does its inner sweeps (PAIR_SWEEP_FLOPS each), and
      every pair checked in a round sums its row-chunk partial Grams (nchunk * 1024 flops);
    k_eig_round (a round's column update fused with the next round's partial Grams): every
      pair's partial Grams over the ld rows (2 ld 32^2 per pair and round) and the column
      update of every pair that rotated (2 ld 32^2)."""
    ld, nblk, npairs, rounds, nchunk = eig_shape(order, tuning.get("gram_rows", GRAM_ROWS))
    real_pairs = nblk // 2 + (nblk & 1)          # the odd block out still solves alone
    inner = tuning.get("inner_sweeps", 1)
    if kernel == "eig_solve":
        return rot * inner * PAIR_SWEEP_FLOPS + sw * rounds * real_pairs * nchunk * 1024
    return sw * rounds * real_pairs * 2.0 * ld * 1024 + rot * 2.0 * ld * 1024


def solve_alg_flops(info, sweeps, rotated, tuning, kernel="eig_solve", routes=None, core=None, mixed=False):
    """Algorithmic flops of the eigensolver launches of `kernel` in one run of a matrix
    (eig_job_flops per core), at the order each core's Jacobi ran on: k for a core on the
    subspace route (its Rayleigh-Ritz matrix), q otherwise (also after a failed check, whose
    Jacobi on G dominates)."""
    tot = 0.0
    cores = ((info["n1"], info["s"], sweeps[1], rotated[0]), (info["s"] + info["n2"], info["r"], sweeps[2], rotated[1]))
    for c, (q, t, sw, rot) in enumerate(cores):
        if q <= 0 or sw <= 0:
            continue
        order = q
        if routes is not None and core is not None and routes[c] == "subspace":
            order = core_basis(core, t, q, mixed) or q
        tot += eig_job_flops(order, sw, rot, tuning, kernel)
    return tot


ROOF_KERNELS = ["cq_panel", "sub_gemm", "eig_round", "eig_solve"]
KERNEL_NAMES = {"cq_panel": "k_cq_panel", "sub_gemm": "k_mfma_gemm (products by G)", "eig_solve": "k_eig_solve",
                "eig_round": "k_eig_round"}


def core_basis(core, t, q, mixed):
    """Basis size of the subspace route (the library's rule, with the factor of the precision
    form), 0 when the core stays on Jacobi."""
    if core["mode"] == 0 or q < core["min_order"] or t <= 0:
        return 0
    k = (int(math.ceil(core["k_factor_mixed" if mixed else "k_factor"] * t)) + 31) // 32 * 32
    return k if (k > t and k <= core["max_frac"] * q) else 0


def kernel_alg_flops(info, routes, core, mixed, tuning, sweeps, rotated):
    """Algorithmic flops per step of the timed kernels.
    sub_gemm: every product Y = G Q of a subspace core, 2 q^2 k each;
    cq_panel: per Cholesky-QR panel launch, the factorisation and inversion of the 64 x 64
      diagonal block (2 * 64^3 / 3) and one 64 x 64 x 64 product (2 * 64^3) for each of the
      kp / 64 - 1 tiles of the panel (its L21 rows and its block row of L^-1);
    eig_round, eig_solve: as eig_job_flops, at the order the Jacobi ran on (k for a subspace
      core's Rayleigh-Ritz matrix, q otherwise)."""
    iters = core["iters_mixed"] if mixed else core["iters_fp64"]
    oe = core["orth_every"]
    out = {"sub_gemm": 0.0, "cq_panel": 0.0, "eig_solve": 0.0, "eig_round": 0.0}
    for c, (q, t) in enumerate(((info["n1"], info["s"]), (info["s"] + info["n2"], info["r"]))):
        if q <= 0 or t <= 0:
            continue
        order = q
        if routes[c] in ("subspace", "subspace+jacobi"):
            k = core_basis(core, t, q, mixed)
            kp = (k + 63) // 64 * 64
            out["sub_gemm"] += iters * 2.0 * q * q * k
            n_orth = (iters + oe - 1) // oe + 2
            out["cq_panel"] += n_orth * (kp // 64) * (2.0 * 64 ** 3 / 3.0 + 2.0 * 64 ** 3 * (kp // 64 - 1))
            order = k
        sw = sweeps[1 + c]
        if sw > 0:
            for kname in ("eig_solve", "eig_round"):
                out[kname] += eig_job_flops(order, sw, rotated[c], tuning, kname)
    return out


def roofline_entry(kname, kms, alg, mixed, config, head_key, core=None, tuning=None):
    """Roofline object of one timed kernel: algorithmic flops per step over its summed launch
    time per step, against the peak of its unit."""
    n_launch, k_ms = kms[kname]
    achieved = alg[kname] / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
    if kname == "sub_gemm":
        bound, peak = "mfma", (157.3 if mixed else 78.6)   # FP32 / FP64 matrix-core peak
    else:
        bound, peak = "alu", 78.6                          # FP64 vector peak
    return {"bound": bound, "kernel": KERNEL_NAMES[kname], "achieved": round(achieved, 5), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 6),
            "traffic": kernel_traffic(kname, config, "mixed" if mixed else "fp64", core, tuning),
            "traffic_unit": "bytes per launch", "launches": round(n_launch, 1),
            "avg_us": round(k_ms / max(n_launch, 1) * 1e3, 3), "ms_per_step": round(k_ms, 4),
            "flops_per_launch": alg[kname] / max(n_launch, 1),
            "timed_in": head_key + " (eager pass of the same schedule)"}


def recon_error(A, U, S, V):
    """||A - U S V^T||_F / ||A||_F via ||A||^2 - 2 tr(S U^T A V) + tr((U^T U) S (V^T V) S)."""
    a2 = float(np.sum(A.data ** 2))
    cross = float(np.sum(S * np.einsum("ij,ij->j", U, A @ V)))
    G = (U.T @ U) * S[None, :]
    H = (V.T @ V) * S[None, :]
    e2 = max(a2 - 2.0 * cross + float(np.sum(G * H.T)), 0.0)
    return math.sqrt(e2 / a2)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_stages(prob, alpha, deadline=None):
    """One run of the oracle, stage by stage (the steps of oracle.fastpi_svd, then the apply),
    with the wall time of each. With a deadline (perf_counter value) no further stage starts
    once it has passed; returns (times, completed)."""
    import oracle
    from oracle.fastpi import block_svd, column_update, row_update, split_blocks
    A = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(prob.m, prob.n))
    A.eliminate_zeros()
    A.sort_indices()
    k = prob.cfg.k
    st = {}
    times = {}

    steps = [
        ("a0_reorder", lambda: st.__setitem__("R", oracle.reorder(prob.m, prob.n, A.indptr, A.indices, k))),
        ("a1_split", lambda: st.__setitem__("S", split_blocks(prob.m, prob.n, A.indptr, A.indices, A.data,
                                                               st["R"]))),
        ("a2_blocks", lambda: st.__setitem__("B", block_svd(st["S"], alpha))),
        ("a3_row_update", lambda: st.__setitem__("R2", row_update(st["S"], st["B"], alpha))),
        ("a4_column_update", lambda: st.__setitem__("R3", column_update(st["S"], st["R2"], alpha,
                                                                         prob.m, prob.n))),
        ("a5_a6_unpermute_apply", lambda: oracle.pinv_apply(
            st["R3"].U[st["R"].piT.astype(np.int64)], st["R3"].sigma,
            st["R3"].V[st["R"].piF.astype(np.int64)], prob.Y, prob.m, prob.n)),
    ]
    for name, fn in steps:
        if deadline is not None and time.perf_counter() >= deadline:
            return times, False
        t0 = time.perf_counter()
        fn()
        times[name] = round(time.perf_counter() - t0, 4)
        progress(f"oracle {name}: {times[name]:.2f} s")
    return times, True


def cpu_baseline(prob, alpha, F, budget_s, full_single):
    """The oracle as it stands on the host cores: one whole run with every thread the BLAS
    library starts (the value, per-stage times), then a single-thread run (the paper times one
    thread), stage by stage, that stops starting stages once budget_s has passed (all stages
    with full_single)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count() or 1
    t0 = time.perf_counter()
    times_n, _ = oracle_stages(prob, alpha)
    dt_n = time.perf_counter() - t0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        times_1, done = oracle_stages(prob, alpha, None if full_single else t0 + budget_s)
        dt_1 = time.perf_counter() - t0
    one = {"cores": 1, "stage_s": times_1, "complete": done}
    if done:
        one["value"] = F / dt_1 / 1e12
        one["s_per_run"] = round(dt_1, 3)
    return {"value": F / dt_n / 1e12, "unit": "TFLOP/s", "cores": int(blas_threads), "kind": "oracle",
            "cpu_model": cpu_model(), "cpus_available": int(avail), "os_cpu_count": os.cpu_count(),
            "stage_s": times_n, "s_per_run": round(dt_n, 3),
            "sample": (f"one whole run of the oracle (reorder, split, block SVDs, both updates, "
                       f"unpermute and apply) on the same workload with {blas_threads} BLAS threads, "
                       f"{dt_n:.1f} s; then one thread, stage by stage"
                       + ("" if done else f", stopped after {len(times_1)} stages at the "
                                          f"{budget_s:.0f} s budget")),
            "single_thread": one}


def run_batched_workload(args, torch, fp):
    """The batched workload: independent matrices of varying shape (synth's sampler). Plain
    form: each matrix on its own handle, one after another, eager launches. Batched form:
    all matrices in one batch (one persistent block-SVD launch, batched eigensolvers,
    graph replay, autotuned schedule). Both apply the pseudoinverse to each matrix's Y."""
    from synth import make_problem, sample_batch_configs
    cfgs = sample_batch_configs(args.batch_count)
    dev = torch.device("cuda", 0)
    probs, plans, F, dev_in = [], [], [], []
    t0 = time.perf_counter()
    for ci_, c in enumerate(cfgs):
        if ci_ % 8 == 0:
            progress(f"generating matrices {ci_}..{min(ci_ + 8, len(cfgs)) - 1}")
        prob = make_problem(c)
        plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=c.alpha, k=c.k)
        F.append(flop_model(plan, plan.blocks(), plan.block_ranks(), c.L, prob.indptr, prob.indices)["total"])
        dev_in.append((torch.from_numpy(prob.indptr).to(dev), torch.from_numpy(prob.indices).to(dev),
                       torch.from_numpy(prob.data).to(dev), torch.from_numpy(prob.Y).to(dev)))
        probs.append(prob)
        plans.append(plan)
    plan_s = time.perf_counter() - t0
    F_tot = float(sum(F))

    def outputs():
        out = []
        for plan, c in zip(plans, cfgs):
            i = plan.info
            out.append((torch.empty((i["m"], i["r"]), dtype=torch.float64, device=dev),
                        torch.empty((i["r"],), dtype=torch.float64, device=dev),
                        torch.empty((i["n"], i["r"]), dtype=torch.float64, device=dev),
                        torch.empty((i["n"], c.L), dtype=torch.float64, device=dev)))
        return out

    def timed(step, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    res = {}
    for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
        progress(f"{prec}: per-matrix runs")
        # plain: one handle per matrix, in sequence
        hs = []
        for plan in plans:
            h = fp.Handle(0, precision=prec)
            h.set_tuning(eig_fused=int(args.eig_rounds == "fused"))
            h.set_core_solver(mode=args.core_mode)
            h.upload_plan(plan)
            hs.append(h)
        outs = outputs()

        def plain_step():
            for h, (rp, ci, va, Y), (U, S, V, Z) in zip(hs, dev_in, outs):
                h.svd(rp, ci, va, out=(U, S, V))
                h.apply(U, S, V, Y, out=Z)

        for _ in range(args.warmup):
            plain_step()
        ms_plain = timed(plain_step, args.steps) * 1e3
        for h in hs:
            h.sync()
        plain_routes = [x for h in hs for x in h.last_core_routes()]
        del hs
        progress(f"{prec}: per-matrix {ms_plain:.1f} ms/step; batched runs (autotune first)")
        # batched: one batch over all matrices on one handle
        h = fp.Handle(0, precision=prec)
        h.set_core_solver(mode=args.core_mode)
        b = fp.Batch(h, plans)
        b.set_tuning(eig_fused=int(args.eig_rounds == "fused"))
        outb = outputs()
        uvs = [(U, S, V) for U, S, V, _ in outb]
        vals = [d[2] for d in dev_in]
        tune_report = b.autotune(vals, out=uvs)
        b.set_graph(True)

        def batched_step():
            b.svd(vals, out=uvs)
            for (rp, ci, va, Y), (U, S, V, Z) in zip(dev_in, outb):
                h.apply(U, S, V, Y, out=Z)

        for _ in range(args.warmup):
            batched_step()
        ms_batched = timed(batched_step, args.steps) * 1e3
        progress(f"{prec}: batched {ms_batched:.1f} ms/step")
        status, sweeps = b.sync()
        rotated = b.rotations()
        routes = b.core_routes()
        core = h.get_core_solver()
        graph_launches = b.last_graph_launches()
        # the dominant kernel, timed in an eager pass of the same schedule
        b.set_graph(False)
        h.timing_start(args.roofline_kernel)
        eager_steps = max(1, args.steps // 2)
        eager_ms = timed(batched_step, eager_steps) * 1e3
        n_launch, k_ms = h.timing_read()
        h.timing_start(None)
        b.set_graph(True)
        # agreement of the two forms (per matrix: largest relative sigma difference)
        sig_diff = 0.0
        sig_nonfinite = 0   # matrices whose comparison is not finite (max() would drop a NaN)
        for o1, o2 in zip(outs, outb):
            s1, s2 = o1[1].cpu().numpy(), o2[1].cpu().numpy()
            keep = s1 > 1e-6 * s1[0]
            rel = np.abs(s1[keep] - s2[keep]) / s1[keep]
            if not np.all(np.isfinite(rel)):
                sig_nonfinite += 1
                continue
            sig_diff = max(sig_diff, float(np.max(rel)) if rel.size else 0.0)
        res[prec] = {"plain_ms": ms_plain, "batched_ms": ms_batched, "eager_batched_ms": eager_ms,
                     "status_ok": int(sum(1 for x in status if x == "OK")),
                     "sweeps_max": sweeps.max(axis=0).tolist(), "tuning": b.get_tuning(),
                     "tune_report": tune_report, "graph_launches_per_step": graph_launches,
                     "n_launch": n_launch, "k_ms": k_ms, "sigma_rel_diff_plain_vs_batched": sig_diff,
                     "sigma_nonfinite_plain_vs_batched": sig_nonfinite,
                     "routes": {r: sum(1 for rr in routes for x in rr if x == r) for r in
                                sorted({x for rr in routes for x in rr})},
                     "plain_routes": {r: plain_routes.count(r) for r in sorted(set(plain_routes))},
                     "solve_alg_flops": eager_steps * sum(
                         solve_alg_flops(plan.info, sw.tolist(), rot.tolist(), b.get_tuning(),
                                         args.roofline_kernel, rr, core, prec == "mixed")
                         for plan, sw, rot, rr in zip(plans, sweeps, rotated, routes))}
        del b, h
    head_key = "mixed" if "mixed" in res else "fp64"
    head = res[head_key]
    ms = head["batched_ms"]
    roof = None
    if head["n_launch"] > 0 and args.roofline_kernel in ("eig_solve", "eig_round"):
        f_alg = head["solve_alg_flops"]
        achieved = f_alg / (head["k_ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": KERNEL_NAMES[args.roofline_kernel], "achieved": round(achieved, 5),
                "peak": 78.6,
                "unit": "TFLOP/s", "frac": round(achieved / 78.6, 6), "traffic": None,
                "launches": head["n_launch"], "avg_us": round(head["k_ms"] / head["n_launch"] * 1e3, 3),
                "flops_per_launch": f_alg / head["n_launch"],
                "timed_in": f"{head_key} batched (eager pass of the same schedule)"}
    base = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = os.cpu_count() or 1
        progress("oracle on the host cores")
        t0 = time.perf_counter()
        done_f = 0.0
        done = 0
        for prob, c, f in zip(probs, cfgs, F):
            r = oracle.fastpi_svd(prob.m, prob.n, prob.indptr, prob.indices, prob.data, c.alpha, c.k)
            oracle.pinv_apply(r.U, r.sigma, r.V, prob.Y, prob.m, prob.n)
            done_f += f
            done += 1
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        dt = time.perf_counter() - t0
        base = {"value": done_f / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
                "sample": f"the oracle on the first {done} of the {len(cfgs)} matrices, in order, "
                          f"{dt:.1f} s"}
    out = {
        "metric": "Ã⁺Y time & TFLOP/s, mixed-precision vs FP64 GPU at equal recon error",
        "value": round(F_tot / (ms * 1e-3) / 1e12, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_key == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"fastpi batched: {len(cfgs)} independent matrices, m 5k-50k, n 500-4k, "
                               "density 0.1-1%, power-law 1.8-2.3, lognormal values, L 100-500, alpha 0.2",
                   "form": f"{head_key}-batched", "matrices": len(cfgs),
                   "nnz_total": int(sum(p.nnz for p in probs))},
        "flop_model_total": F_tot,
        "plan_s": round(plan_s, 3),
        # times to 4 decimals; the sigma agreement keeps its significant digits (it sits near 1e-13)
        "forms": {k: {kk: (float(f"{vv:.3g}") if kk.startswith("sigma_") else round(vv, 4))
                      if isinstance(vv, float) else vv for kk, vv in v.items()}
                  for k, v in res.items()},
        "speedup_batched_vs_plain": {k: round(v["plain_ms"] / v["batched_ms"], 4) for k, v in res.items()},
        "roofline": roof,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


def run_eval_workload(args, torch, fp):
    """Application 1's evaluation loop on the labelled form of a workload (planted labels,
    90/10 row split; synth.make_labelled_problem): the SVD of the training rows once, then
    per step the sparse-label apply Z = V Sigma^+ U^T Y and the top-k hit counts of the test
    rows. The dense-label apply of the same Y is timed beside it."""
    import oracle
    from synth import CONFIGS, make_labelled_problem
    cfg = CONFIGS[args.config]
    progress(f"generating labelled {args.config}")
    lp = make_labelled_problem(cfg)
    tr, te, L = lp.train, lp.test, lp.L
    precision = "mixed" if args.precision == "mixed" else "fp64"
    dev = torch.device("cuda", 0)
    plan = fp.Plan(tr.m, tr.n, tr.indptr, tr.indices, tr.data, alpha=cfg.alpha, k=cfg.k)
    info = plan.info
    m, n, r = info["m"], info["n"], info["r"]
    h = fp.Handle(0, precision=precision)
    h.upload_plan(plan)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    progress(f"SVD of the training rows {m}x{n} (r={r})")
    U, S, V = h.svd(t(tr.indptr), t(tr.indices), t(tr.data))
    h.sync()
    t0 = time.perf_counter()
    labels = fp.Labels(h, m, L, tr.y_indptr, tr.y_indices)
    labels_s = time.perf_counter() - t0
    Yd = t(oracle.labels_dense(m, L, tr.y_indptr, tr.y_indices))
    te_in = [t(a) for a in (te.indptr, te.indices, te.data)]
    ty_in = [t(a) for a in (te.y_indptr, te.y_indices)]
    ks = [1, 3, 5]
    Z = torch.empty((n, L), dtype=torch.float64, device=dev)
    hits = torch.empty((te.m, len(ks)), dtype=torch.int32, device=dev)

    def time_calls(fn, kernels):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        per = {}
        for kname in kernels:
            h.timing_start(kname)
            for _ in range(args.steps):
                fn()
            per[kname] = h.timing_read()
        h.timing_start(None)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, per

    progress("timing the sparse-label apply, the dense-label apply and the scoring")
    sp_ms, sp_k = time_calls(lambda: h.apply_sparse(U, S, V, labels, out=Z), ["label_spmm", "gemm_nt"])
    dn_ms, _ = time_calls(lambda: h.apply(U, S, V, Yd), [])
    h.apply_sparse(U, S, V, labels, out=Z)
    tk_ms, tk_k = time_calls(lambda: h.topk_hits(*te_in, Z, *ty_in, ks, out=hits), ["topk"])
    hits_h = hits.cpu().numpy().astype(np.int64)
    p_at = oracle.p_at_k(hits_h, ks)
    kern = {}
    for name, (cnt, ms_tot) in {**sp_k, **tk_k}.items():
        kern[name] = {"launches": cnt, "avg_us": round(ms_tot / max(cnt, 1) * 1e3, 3)}
    # algorithmic bytes of the label SpMM: the U rows that carry a label, Y^T's entries
    # (row id and value), the L x r product written once
    rows_with_label = int(np.count_nonzero(np.diff(tr.y_indptr)))
    spmm_bytes = rows_with_label * r * 8 + tr.y_nnz * 12 + L * r * 8
    spmm_launch_us = sp_k["label_spmm"][1] / max(args.steps, 1) * 1e3   # both passes, per call
    achieved = spmm_bytes / (spmm_launch_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": "k_label_spmm (+ k_label_reduce)", "achieved": round(achieved, 2),
            "peak": 8000.0, "unit": "GB/s", "frac": round(achieved / 8000.0, 5),
            "traffic": label_spmm_traffic(args.config), "traffic_unit": "bytes per call",
            "bytes_per_call": spmm_bytes, "us_per_call": round(spmm_launch_us, 3)}
    base = None
    if not args.no_cpu_baseline:
        progress("oracle on the host cores (apply and scoring)")
        Uh, Sh, Vh = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        c0 = time.perf_counter()
        Zo = oracle.pinv_apply_sparse(Uh, Sh, Vh, m, n, L, tr.y_indptr, tr.y_indices)
        c1 = time.perf_counter()
        rows = min(te.m, 2000)
        sub_ptr = te.indptr[:rows + 1]
        oracle.topk_hits(sub_ptr, te.indices, te.data, Zo, te.y_indptr[:rows + 1], te.y_indices, ks)
        c2 = time.perf_counter()
        cpu_ms = (c1 - c0) * 1e3 + (c2 - c1) * 1e3 * te.m / rows
        base = {"value": round(cpu_ms, 3), "unit": "ms per evaluation", "cores": int(torch.get_num_threads()),
                "kind": "oracle",
                "sample": f"one oracle apply of the full Y and scoring of {rows} of {te.m} test rows "
                          f"({c2 - c0:.1f} s), scoring scaled to all rows"}
    out = {
        "metric": "evaluation loop time (sparse-label apply + top-k scoring of the test rows)",
        "value": round(sp_ms + tk_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sp_ms + tk_ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"fastpi {cfg.name} labelled: train {m}x{n} ({tr.nnz} nnz), "
                               f"Y {m}x{L} ({tr.y_nnz} positives), test {te.m} rows, alpha {cfg.alpha}",
                   "r": r, "ks": ks},
        "apply_sparse_ms": round(sp_ms, 4),
        "apply_dense_ms": round(dn_ms, 4),
        "speedup_sparse_vs_dense_apply": round(dn_ms / sp_ms, 3),
        "topk_ms": round(tk_ms, 4),
        "kernels": kern,
        "labels_upload_s": round(labels_s, 4),
        "p_at_k": {str(k): round(float(v), 5) for k, v in zip(ks, p_at)},
        "roofline": roof,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


def run_reorder_workload(args, torch, fp):
    """Algorithm 2 on the GPU (fastpi_reorder_gpu on the device CSR) against the host
    reordering, on the same pattern: one warm-up call, then the median of --steps calls; the
    two results must be identical."""
    from synth import CONFIGS, make_problem
    cfg = CONFIGS[args.config]
    progress(f"generating {args.config}")
    prob = make_problem(cfg)
    dev = torch.device("cuda", 0)
    h = fp.Handle(0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    dargs = (prob.m, prob.n, t(prob.indptr), t(prob.indices), t(prob.data))
    gpu = h.reorder(*dargs, k=cfg.k)
    times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gpu = h.reorder(*dargs, k=cfg.k)
        times.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    host = fp.reorder(prob.m, prob.n, prob.indptr, prob.indices, prob.data, k=cfg.k)
    host_s = time.perf_counter() - t0
    same = all(np.array_equal(a, b) for a, b in zip(host[:3], gpu[:3])) and host[3] == gpu[3]
    ms = sorted(times)[len(times) // 2] * 1e3
    out = {
        "metric": "reordering time (Algorithm 2), GPU vs host, identical output",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": len(times), "warmup": 1,
        "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"fastpi {cfg.name}: A {prob.m}x{prob.n} ({prob.nnz} nnz), k {cfg.k}",
                   "T_it": gpu[3]["T_it"], "blocks": int(len(gpu[2]))},
        "host_ms": round(host_s * 1e3, 3), "identical": bool(same),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--form", default="both", choices=["plain", "batched", "both"])
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds after which the single-thread oracle run starts no further stage")
    ap.add_argument("--cpu-full-single", action="store_true",
                    help="run every stage of the single-thread oracle, whatever its time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-kernel", default="eig_round",
                    choices=["eig_round", "eig_solve", "eig_gram", "eig_update", "block_svd", "cq_panel", "sub_gemm"],
                    help="kernel timed for the roofline of the batched 64-matrix workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (scale for the PMC byte counters)")
    ap.add_argument("--batch-count", type=int, default=64, help="matrices of the batched workload")
    ap.add_argument("--eig-rounds", default="fused", choices=["fused", "three"],
                    help="eigensolver rounds: two launches each (column update fused with the next "
                         "round's partial Grams, then the pair solves; default) or three")
    ap.add_argument("--block-route", type=float, default=None,
                    help="p q^2 from which a diagonal block takes the Gram route (default: the library's)")
    ap.add_argument("--gram-rows", type=int, default=None, choices=[64, 128, 256],
                    help="rows per partial Gram of the eigensolvers (plain form; default: the library's)")
    ap.add_argument("--eig-precond", type=int, default=None, choices=[0, 1],
                    help="pivoted-Cholesky start of the core and Rayleigh-Ritz eigensolves (plain form; "
                         "default: the library's)")
    ap.add_argument("--core-mode", type=int, default=1, choices=[0, 1],
                    help="core solver of the updates: 0 block Jacobi on G, 1 subspace iteration where it applies")
    ap.add_argument("--core-max-frac", type=float, default=None,
                    help="largest basis-to-order ratio k/q of the subspace route (default: the library's)")
    ap.add_argument("--core-min-order", type=int, default=None,
                    help="smallest core order q of the subspace route (default: the library's)")
    ap.add_argument("--core-k-factor", type=float, default=None,
                    help="basis of the subspace route in the form being run, k = ceil32(factor * t) "
                         "(default: the library's)")
    ap.add_argument("--core-orth-every", type=int, default=None,
                    help="products by G between Cholesky QRs of the subspace route (default: the library's)")
    ap.add_argument("--core-iters", type=int, default=None,
                    help="products by G of the subspace route in the form being run (default: the library's)")
    ap.add_argument("--inner", default="exact", choices=["exact", "rand"],
                    help="inner solver of the two updates: exact, or the randomized branch where "
                         "the target rank is low (oversampling 5, 11 power iterations)")
    ap.add_argument("--reorder", action="store_true",
                    help="time the GPU reordering against the host one on the workload's pattern")
    ap.add_argument("--eval", action="store_true",
                    help="time Application 1's evaluation loop (sparse-label apply + P@k scoring)")
    ap.add_argument("--ranks", default="alpha", choices=["alpha", "learned"],
                    help="block ranks: the alpha rule, or the shipped rank network at the same total")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2011_04235_amd as fp
    from synth import CONFIGS, make_problem

    if args.calibrate_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.config == "c4":
        return run_batched_workload(args, torch, fp)
    if args.eval:
        return run_eval_workload(args, torch, fp)
    if args.reorder:
        return run_reorder_workload(args, torch, fp)

    cfg = CONFIGS[args.config]
    progress(f"generating {args.config}")
    prob = make_problem(cfg)
    progress(f"planning {prob.m}x{prob.n}, {prob.nnz} nonzeros")
    fp.load()
    t0 = time.perf_counter()
    plan = fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=cfg.alpha, k=cfg.k)
    plan_s = time.perf_counter() - t0
    # the same plan with the reordering on the GPU (one warm-up call, then the median of three)
    hr = fp.Handle(0)
    fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=cfg.alpha, k=cfg.k, gpu=hr)
    gpu_plan_times = []
    for _ in range(3):
        t0 = time.perf_counter()
        fp.Plan(prob.m, prob.n, prob.indptr, prob.indices, prob.data, alpha=cfg.alpha, k=cfg.k, gpu=hr)
        gpu_plan_times.append(time.perf_counter() - t0)
    plan_gpu_s = sorted(gpu_plan_times)[1]
    del hr
    ranks_note = "alpha rule"
    if args.ranks == "learned":
        from paper_2011_04235_amd.rank_mlp import RankPredictor
        pred = RankPredictor.load(os.path.join(ROOT, "paper_2011_04235_amd", "rank_predictor.npz"))
        feats = plan.block_features(prob.data)
        hk = fp.Handle(0)
        plan.set_block_ranks(pred.block_ranks(hk, plan, prob.data))
        del hk
        ranks_note = (f"rank network ({int(pred.in_range(feats).sum())} of {len(feats)} blocks; the rest "
                      "alpha rule), total s_b of the alpha rule")
    blocks = plan.blocks()
    ranks = plan.block_ranks()
    F = flop_model(plan, blocks, ranks, cfg.L, prob.indptr, prob.indices)

    dev = torch.device("cuda", 0)
    rowptr = torch.from_numpy(prob.indptr).to(dev)
    col = torch.from_numpy(prob.indices).to(dev)
    val = torch.from_numpy(prob.data).to(dev)
    Y = torch.from_numpy(prob.Y).to(dev)
    m, n, r = plan.m, plan.n, plan.r
    A_host = sp.csr_matrix((prob.data, prob.indices, prob.indptr), shape=(m, n))

    def run_path(precision, batched):
        """Plain form: eager launches with the default schedule. Batched form: the
        autotuned schedule and the stage chain replayed from HIP graphs."""
        progress(f"{precision} {'batched' if batched else 'plain'}: start")
        h = fp.Handle(0, precision=precision)
        h.set_tuning(eig_fused=int(args.eig_rounds == "fused"),
                     **({"precond": args.eig_precond} if args.eig_precond is not None else {}),
                     **({"gram_rows": args.gram_rows} if args.gram_rows is not None else {}))
        h.set_core_solver(mode=args.core_mode,
                          **({"max_frac": args.core_max_frac} if args.core_max_frac is not None else {}),
                          **({"min_order": args.core_min_order} if args.core_min_order is not None else {}),
                          **({("k_factor_mixed" if precision == "mixed" else "k_factor"): args.core_k_factor}
                             if args.core_k_factor is not None else {}),
                          **({("iters_mixed" if precision == "mixed" else "iters_fp64"): args.core_iters}
                             if args.core_iters is not None else {}),
                          **({"orth_every": args.core_orth_every} if args.core_orth_every is not None else {}))
        if args.inner == "rand":
            h.set_inner(mode=1, oversample=5, iters=11, seed=0)
        if args.block_route is not None:
            h.set_block_route(args.block_route)
        h.upload_plan(plan)
        U = torch.empty((m, r), dtype=torch.float64, device=dev)
        S = torch.empty((r,), dtype=torch.float64, device=dev)
        V = torch.empty((n, r), dtype=torch.float64, device=dev)
        Z = torch.empty((n, cfg.L), dtype=torch.float64, device=dev)
        tune_report = None
        if batched:
            tune_report = h.autotune(rowptr, col, val, out=(U, S, V))
            progress(f"  autotuned: {tune_report.split('chose')[-1].strip()}")
            h.set_graph(True)

        def step():
            h.svd(rowptr, col, val, out=(U, S, V))
            h.apply(U, S, V, Y, out=Z)

        def timed(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                step()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / k

        for _ in range(args.warmup):
            step()
        h.sync()
        dt = timed(args.steps)
        h.sync()
        progress(f"  timed {args.steps} steps: {dt * 1e3:.2f} ms/step")
        graph_launches = h.last_graph_launches()
        sweeps = h.last_sweeps()
        rotated = h.last_rotations()
        routes = h.last_core_routes()
        # candidate kernels timed launch by launch with HIP events on the library's stream, in
        # eager passes of the same schedule right after the timed region (graph replays carry
        # no per-kernel events); each pass runs `kpass` steps
        kernel_ms = {}
        if batched:
            h.set_graph(False)
        eager_dt = None
        kpass = max(2, args.steps // 2)
        for kname in ROOF_KERNELS:
            h.timing_start(kname)
            edt = timed(kpass)
            n_launch, k_ms = h.timing_read()
            kernel_ms[kname] = (n_launch / kpass, k_ms / kpass)
            eager_dt = edt if eager_dt is None else min(eager_dt, edt)
        h.timing_start(None)
        if batched:
            h.set_graph(True)
        Uh, Sh, Vh = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        out = {"ms": dt * 1e3, "sweeps": sweeps, "rotated": rotated, "kernel_ms": kernel_ms,
               "routes": routes, "core": h.get_core_solver(),
               "recon": recon_error(A_host, Uh, Sh, Vh), "sigma": Sh, "tuning": h.get_tuning(),
               "graph_launches_per_step": graph_launches}
        if batched:
            out["tune_report"] = tune_report
        out["eager_ms"] = eager_dt * 1e3
        return out

    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    forms = {"plain": False, "batched": True} if args.form == "both" else {args.form: args.form == "batched"}
    res = {f"{p}-{f}": run_path(p, b) for p in precs for f, b in forms.items()}
    head_key = [k for k in ("mixed-batched", "mixed-plain", "fp64-batched", "fp64-plain") if k in res][0]
    head = res[head_key]
    ms = head["ms"]
    tflops = F["total"] / (ms * 1e-3) / 1e12
    sweeps = head["sweeps"]
    mixed_head = head_key.startswith("mixed")
    alg = kernel_alg_flops(plan.info, head["routes"], head["core"], mixed_head, head["tuning"], sweeps,
                           head["rotated"])
    kms = head["kernel_ms"]
    share = {k: round(v[1] / head["eager_ms"], 4) for k, v in kms.items()}
    # the dominant kernel: the largest summed launch time per step among the timed ones
    dom = max((k for k in kms if kms[k][0] > 0), key=lambda k: kms[k][1], default=None)
    roof = roofline_entry(dom, kms, alg, mixed_head, args.config, head_key, head["core"], head["tuning"]) \
        if dom else None
    roof_mfma = roofline_entry("sub_gemm", kms, alg, mixed_head, args.config, head_key, head["core"],
                               head["tuning"]) \
        if kms.get("sub_gemm", (0, 0))[0] > 0 else None
    base = None
    if not args.no_cpu_baseline:
        progress("oracle on the host cores")
        base = cpu_baseline(prob, cfg.alpha, F["total"], args.cpu_budget, args.cpu_full_single)
    compare = {p: {"ms_per_step": round(v["ms"], 3), "tflops": round(F["total"] / v["ms"] / 1e9, 4),
                   "recon_error": v["recon"], "sweeps": v["sweeps"], "tuning": v["tuning"],
                   "graph_launches_per_step": v["graph_launches_per_step"],
                   "core_routes": v["routes"],
                   "kernel_ms_per_step": {k: round(x[1], 4) for k, x in v["kernel_ms"].items()},
                   "eager_ms_per_step": round(v["eager_ms"], 3),
                   **({"tune_report": v["tune_report"]} if "tune_report" in v else {})}
               for p, v in res.items()}
    ref_key = "fp64-plain" if "fp64-plain" in res else None
    if ref_key:
        ref = res[ref_key]
        for k, v in res.items():
            if k == ref_key:
                continue
            compare[f"speedup_{k}_vs_{ref_key}"] = round(ref["ms"] / v["ms"], 4)
            compare[f"recon_error_diff_{k}"] = abs(ref["recon"] - v["recon"])
            s64, sx = ref["sigma"], v["sigma"]
            keep = s64 > 1e-6 * s64[0]
            compare[f"sigma_rel_diff_{k}"] = float(np.max(np.abs(s64[keep] - sx[keep]) / s64[keep]))

    # the path's roofline time by the flop model's stages, T_roof = sum max(F_i / P_i, B_i / BW):
    # the gather's bytes (a1), each stage's flops at the peak of its precision (mixed: the block
    # Jacobi and the apply in FP32, the two updates' cores in FP64), frac = T_roof / T_path
    blocks_dense = blocks[(blocks[:, 2] > 0) & (blocks[:, 3] > 0)]
    b1 = (prob.nnz * 12 + (m + 1) * 8 + (m + n) * 4 + float(np.sum(blocks_dense[:, 2] * blocks_dense[:, 3])) * 8
          + F["nnz_A21"] * 12 + F["nnz_T"] * 12)
    mixed_head_form = head_key.startswith("mixed")
    p32, p64, bw = 157.3e12, 78.6e12, 8.0e12
    t_roof = (b1 / bw + F["a2"] / (p32 if mixed_head_form else p64) + F["a3"] / p64 + F["a4"] / p64
              + max(F["a6"] / (p32 if mixed_head_form else p64), 8.0 * (m * cfg.L + m * r + n * r + n * cfg.L) / bw))
    path_roof = {"t_roof_ms": round(t_roof * 1e3, 4), "t_path_ms": round(ms, 4), "frac": round(t_roof * 1e3 / ms, 4),
                 "basis": "flop model stages at the MI355X peaks of their precision (a1 at HBM 8 TB/s)"}

    out = {
        "metric": "Ã⁺Y time & TFLOP/s, mixed-precision vs FP64 GPU at equal recon error",
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_key.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": f"fastpi {cfg.name}: A {m}x{n} ({prob.nnz} nnz, power-law "
                               f"{cfg.gamma}, {cfg.values}), Y {m}x{cfg.L}, alpha {cfg.alpha}",
                   "form": head_key, "ranks": ranks_note, "inner": args.inner, "m": m, "n": n,
                   "nnz": prob.nnz, "L": cfg.L,
                   "alpha": cfg.alpha, "shape": plan.info},
        "flop_model": F,
        "plan_s": round(plan_s, 4),
        "plan_gpu_reorder_s": round(plan_gpu_s, 4),
        "sweeps": sweeps,
        "precision_compare": compare,
        "roofline": roof,
        "roofline_mfma": roof_mfma,
        "path_roofline": path_roof,
        "kernel_share_of_eager_step": share,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

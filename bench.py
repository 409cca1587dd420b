#!/usr/bin/env python3
"""Benchmark of the Epstein-zeta hot path on one MI355X.

Workload (one step): the ATM cohesive energy per particle of the sc, fcc and
bcc lattices at unit density, d = 3, FP64, each on a 263424-node plan
(12 Duffy blocks x 14^2 Gauss-Legendre v-nodes x 112 u-nodes on 7 geometric
panels toward k = 0, plus the Taylor/Hadamard part on (0, 1e-2)).  One step
is one ez_atm_energy call on the batch of three generator matrices already
resident in HBM: lattice tables, nodes, reciprocal and real-space sums,
singular split, products, Hadamard part and fixed-order reduction.

Prints one JSON line.  `value` = ATM lattice sums per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP64_MFMA_TFLOPS = 78.6     # MI355X published dense FP64 matrix peak
METRIC = "ATM lattice sums/s and Epstein-zeta evals/s at 1e-12 rel err, FP64 vs mixed"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nodes_c2.json")
KERNEL_SOURCES = ["ez_nodes.hip", "ez_quad_common.h", "ez_math.h", "ez_internal.h", "ez_kernels.h", "e1_rational.h",
                  "exp2_table.h", "ep_f32_rational.h"]


def node_kernel_flops_per_node(lam_rel: float, a_cut: float, n_nu: int, d: int = 3) -> float:
    """Algorithmic FP64 flops of one quadrature node (unit-density lattice), FMA = 2:
    N_rec reciprocal terms x (8 for |m*+k|^2, 70 for exp + E1, 7.5 per exponent for
    the E_p recurrence and accumulation) + N_real real-space pairs x (6 for the
    complex rotation that advances e^{2 pi i k.z} + 2 per exponent), with
    N_rec = |ball of radius sqrt(a_cut/pi)/lam| and N_real = |ball of radius
    lam sqrt(a_cut/pi)| / 2 (lattice and reciprocal lattice of unit covolume)."""
    import math
    r = math.sqrt(a_cut / math.pi)
    ball = {1: 2.0, 2: math.pi, 3: 4.0 * math.pi / 3.0}[d]
    n_rec = ball * (r / lam_rel) ** d
    n_real = 0.5 * ball * (r * lam_rel) ** d
    rec_term = 8.0 + 70.0 + 7.5 * n_nu
    real_term = 6.0 + 2.0 * n_nu
    return n_rec * rec_term + n_real * real_term


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_11989_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, min_seconds: float = 10.0) -> dict:
    """The oracle (oracle/ezo.c, OpenMP over directions) on the same three
    lattices at the full plan, sc, fcc, bcc in turn, repeated until at least
    min_seconds of work (a bounded sample of the timed workload), with all the
    host threads; then one lattice sum (sc) on a single thread."""
    import oracle
    import workloads as W
    lats = [W.sc(), W.fcc(), W.bcc()]
    n_all = oracle.num_threads()
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.atm(lats[n % 3], spec)
        n += 1
        dt = time.perf_counter() - t0
        if n >= 3 and dt >= min_seconds:
            break
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.atm(lats[0], spec)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(n_all)
    return {"value": n / dt, "unit": "ATM lattice sums/s", "cores": n_all, "kind": "oracle",
            "sample": "%d lattice sums (sc, fcc, bcc in turn), full 263424-node plan each, %.1f s" % (n, dt),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": 1.0 / dt1, "unit": "ATM lattice sums/s", "cores": 1,
                              "sample": "1 lattice sum (sc), full plan, %.1f s" % dt1}}


def c3_scan_leg(args) -> dict:
    """Batched scan: 4096 body-centred-tetragonal lattices (c/a ~ U[0.8, 1.6], unit
    density, seed 3) with uneven plans of about n^3 nodes, n ~ U{16..64}; per lattice
    the ATM energy and zeta^(3)(nu,nu,nu) for nu in {3, 6, 9, 12}, one node set.
    Plain form: one eager call at lam = 1 with one workgroup per tile.  Chosen form:
    lam and node-kernel schedule from the autotuner (on a 512-lattice sample), the
    call captured into a HIP graph and replayed."""
    import numpy as np
    import torch

    import oracle
    import workloads as W
    from paper_2504_11989_amd import autotune
    from paper_2504_11989_amd.batch import SCAN_NU, SCAN_RESULTS, SCAN_TERMS, GraphedLatticeSums, scan_sums

    ca, nside, A_np = W.c3_scan()
    specs = [W.c3_spec(int(n)) for n in nside]
    nodes = sum(W.n_nodes(3, sp) for sp in specs)
    A = torch.tensor(A_np, dtype=torch.float64, device="cuda")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    plain_specs = autotune.apply(specs, 1.0, 0)
    t_plain = timed(lambda: scan_sums(A, plain_specs), args.c3_reps)
    sample = slice(0, 512)
    tuned = autotune.tune(A[sample], SCAN_NU, SCAN_TERMS, len(SCAN_RESULTS), specs[sample], reps=2,
                          wave_shapes=autotune.DEFAULT_WAVE_SHAPES)
    chosen = autotune.apply(specs, tuned["lam"], tuned["flags"])
    g = GraphedLatticeSums(A, SCAN_NU, SCAN_TERMS, len(SCAN_RESULTS), chosen)
    t_graph = timed(g.replay, args.c3_reps)
    # node-kernel time of one eager call at the chosen configuration (library HIP
    # events on the launch stream) for the roofline: the model's FP64 flops per
    # node (seven exponents) over every node of the batch
    from paper_2504_11989_amd import _native as nat
    scan_sums(A, chosen)
    torch.cuda.synchronize()
    nat.timing_reset()
    nat.timing_enable(True)
    for _ in range(2):
        scan_sums(A, chosen)
    torch.cuda.synchronize()
    nat.timing_enable(False)
    kn = nat.timing_read(nat.KERNEL_NODES)
    node_ms = kn[0] / max(1, kn[1])
    flops = sum(node_kernel_flops_per_node(sp["lam"], sp["a_cut"], len(SCAN_NU)) * W.n_nodes(3, sp)
                for sp in chosen)
    achieved = flops / (node_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 5), "traffic": None,
                "kernel": "ez_node_kernel<3,7,4>", "kernel_ms": round(node_ms, 4), "flops_per_launch": flops}
    out = g.out.cpu().numpy()
    st = g.status.cpu().numpy()
    plain = scan_sums(A, plain_specs).cpu().numpy()
    # parity: the oracle on the three smallest plans, every result, with the chosen lam
    idx = [int(i) for i in np.argsort(nside, kind="stable")[:3]]
    err = 0.0
    for i in idx:
        sp = chosen[i]
        ref = [oracle.atm(A_np[i], sp)] + [oracle.nbody(A_np[i], [nu] * 3, sp) for nu in (3.0, 6.0, 9.0, 12.0)]
        err = max(err, max(abs(out[i, r] - ref[r]) / abs(ref[r]) for r in range(5)))
    return {
        "workload": "4096 bct lattices, c/a ~ U[0.8,1.6], unit density, plans ~n^3 nodes with n ~ U{16..64} "
                    "(seed 3); results: E_ATM and zeta3(nu,nu,nu), nu in {3,6,9,12}; FP64",
        "lattices": len(specs), "nodes_total": int(nodes),
        "lattices_per_s": len(specs) / t_graph, "ms_per_pass": 1e3 * t_graph,
        "epstein_evals_per_s": nodes * len(SCAN_NU) / t_graph,
        "plain": {"form": "eager call, lam = 1, one workgroup per tile", "ms_per_pass": 1e3 * t_plain,
                  "lattices_per_s": len(specs) / t_plain},
        "chosen": {"form": "autotuned lam and schedule, HIP-graph replay", "lam": tuned["lam"],
                   "schedule": tuned["schedule"], "wave_block": tuned["wave"],
                   "tuning_table_ms": [[l, n, w, round(m, 3)] for l, n, w, m in tuned["table"]]},
        "speedup_vs_plain": t_plain / t_graph,
        "max_rel_diff_chosen_vs_plain": float(np.max(np.abs(out - plain) / np.abs(plain))),
        "max_rel_err_vs_oracle_sample": err, "oracle_sample": idx,
        "status_nonzero": int(np.count_nonzero(st)),
        "roofline": roofline,
    }


def c4_grid_leg(args) -> dict:
    """Mixed precision: Z_nu(x_j, y_m) for nu in {-1, 1, 3, 5}, 512 shifts x uniform in the
    cell (seed 4) and 8192 points y uniform in the reciprocal cell (seed 40), on each
    of the sc/fcc/bcc lattices at unit density: 16.8 M Epstein evaluations per lattice,
    as FP64 matrix products (plain) and with the far table entries as split-BF16
    products (mixed).  Errors: mixed against FP64 over the whole grid, both against
    the oracle at 16 sampled (x, y) pairs per lattice."""
    import numpy as np
    import torch

    import oracle
    import workloads as W
    import paper_2504_11989_amd as ez

    nu = [-1.0, 1.0, 3.0, 5.0]
    out = {"workload": "Z_nu(x_j, y_m), nu in {-1,1,3,5}, 512 shifts (seed 4) x 8192 reciprocal-cell points "
                       "(seed 40), sc/fcc/bcc at unit density", "lattices": {}}
    tot = {False: 0.0, True: 0.0}
    worst = {"mixed_vs_fp64": 0.0, "fp64_vs_oracle": 0.0, "mixed_vs_oracle": 0.0, "bound_max": 0.0, "bound_rel": 0.0}
    rng = np.random.default_rng(7)
    from paper_2504_11989_amd import _native as nat
    gemm = {"ms": 0.0, "flops": 0.0, "tables": {}}
    for name, A_np in W.c2_lattices().items():
        A = torch.tensor(A_np, device="cuda")
        xs_np, ys_np = W.c4_shifts(A_np), W.c4_points(A_np)
        xs, ys = torch.tensor(xs_np, device="cuda"), torch.tensor(ys_np, device="cuda")
        res = {}
        for mixed in (False, True):
            ez.epstein_grid(A, nu, xs, ys, mixed=mixed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.c4_reps):
                z = ez.epstein_grid(A, nu, xs, ys, mixed=mixed, with_bound=mixed)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.c4_reps
            tot[mixed] += dt
            res[mixed] = (z, dt)
        # the FP64 products (library HIP events on the launch stream) for the roofline
        nat.timing_reset()
        nat.timing_enable(True)
        for _ in range(2):
            ez.epstein_grid(A, nu, xs, ys)
        torch.cuda.synchronize()
        nat.timing_enable(False)
        gm, gn = nat.timing_read(nat.KERNEL_GRID_GEMM)
        nr, nk = nat.grid_last_tables()
        gemm["ms"] += gm / max(1, gn)
        gemm["flops"] += 4.0 * len(nu) * xs_np.shape[0] * ys_np.shape[0] * (nr + nk)
        gemm["tables"][name] = [nr, nk]
        z64 = res[False][0]
        zm, bound = res[True][0]
        err = ((zm - z64).abs() / z64.abs().clamp(min=1.0)).max().item()
        # the bound at (nu, x_j, y_m) is a shift term plus a point term; in the measure of
        # the comparisons below it is the certified relative error
        nx = xs_np.shape[0]
        bfull = bound[:, :nx, None] + bound[:, None, nx:]
        bmax = bfull.max().item()
        brel = (bfull / zm.abs().clamp(min=1.0)).max().item()
        del bfull
        idx = [(int(rng.integers(512)), int(rng.integers(8192))) for _ in range(16)]
        e64 = em = 0.0
        for j, m in idx:
            for k, v in enumerate(nu):
                ref = oracle.epstein(A_np, v, xs_np[j], ys_np[m])
                den = max(abs(ref), 1.0)
                e64 = max(e64, abs(z64[k, j, m].item() - ref) / den)
                em = max(em, abs(zm[k, j, m].item() - ref) / den)
        worst["mixed_vs_fp64"] = max(worst["mixed_vs_fp64"], err)
        worst["fp64_vs_oracle"] = max(worst["fp64_vs_oracle"], e64)
        worst["mixed_vs_oracle"] = max(worst["mixed_vs_oracle"], em)
        worst["bound_max"] = max(worst["bound_max"], bmax)
        worst["bound_rel"] = max(worst["bound_rel"], brel)
        out["lattices"][name] = {"fp64_ms": 1e3 * res[False][1], "mixed_ms": 1e3 * res[True][1]}
        del z64, zm, bound, res
    evals = 3 * len(nu) * 512 * 8192
    out.update({
        "epstein_evals_per_s_fp64": evals / tot[False], "epstein_evals_per_s_mixed": evals / tot[True],
        "speedup_mixed_vs_fp64": tot[False] / tot[True],
        "max_err_mixed_vs_fp64": worst["mixed_vs_fp64"], "max_err_fp64_vs_oracle": worst["fp64_vs_oracle"],
        "max_err_mixed_vs_oracle": worst["mixed_vs_oracle"], "max_a_priori_bound_mixed": worst["bound_max"],
        "max_a_priori_bound_mixed_rel": worst["bound_rel"],
        # FP64 matrix products: algorithmic flops 2 M N K of the two products per call,
        # (n_nu n_x) x (2 n_y) x n_real and (2 n_x) x (n_nu n_y) x n_rec, summed over the
        # three lattices, over the summed per-call product time
        "roofline": {"bound": "mfma", "achieved": round(gemm["flops"] / (gemm["ms"] * 1e-3) / 1e12, 4),
                     "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(gemm["flops"] / (gemm["ms"] * 1e-3) / 1e12 / PEAK_FP64_MFMA_TFLOPS, 5),
                     "traffic": None, "kernel": "gemm_mixed_kernel<false> (FP64 MFMA, both products)",
                     "kernel_ms_per_call": round(gemm["ms"] / 3, 4), "tables_real_rec": gemm["tables"]},
        "error_measure": "|dZ| / max(|Z|, 1) per element; the a-priori bound per element, absolute and over "
                         "max(|Z|, 1)"})
    return out


def mixed_leg(args, A, spec, gold, names, ms_fp64, node_ms_fp64) -> dict:
    """The three-lattice ATM step in mixed precision (far-field reciprocal terms in
    FP32, bound per result) against the FP64 step, for several FP32 thresholds
    a_mix; `chosen` is the fastest a_mix whose bound certifies 1e-10 relative."""
    import numpy as np
    import torch
    import paper_2504_11989_amd as ez
    from paper_2504_11989_amd import _native as nat
    atm_nu = [-1.0, 1.0, 3.0, 5.0]
    atm_terms = [(0, 1.0 / 24.0, [(2, 3)]), (0, -3.0 / 16.0, [(0, 1), (3, 2)]),
                 (0, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)])]
    v64 = ez.atm_energy(A, spec).cpu().numpy()
    ref = np.array([gold["atm"][n] for n in names])
    table = []
    steps = max(1, args.steps)
    for a_mix in (8, 12, 16, 20, 24):
        sm = dict(spec, precision=nat.PREC_MIXED, flags=nat.spec_mix_a(a_mix))
        for _ in range(max(1, args.warmup)):
            ez.atm_energy(A, sm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ez.atm_energy(A, sm)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        nat.timing_reset()
        nat.timing_enable(True)
        for _ in range(min(steps, 30)):
            ez.atm_energy(A, sm)
        torch.cuda.synchronize()
        nat.timing_enable(False)
        kn = nat.timing_read(nat.KERNEL_NODES)
        v, bd = ez.lattice_sums(A, atm_nu, atm_terms, 1, sm, with_bound=True)
        v, bd = v.cpu().numpy()[:, 0], bd.cpu().numpy()[:, 0]
        table.append({"a_mix": a_mix, "ms_per_step": round(ms, 5), "node_kernel_ms": round(kn[0] / max(1, kn[1]), 5),
                      "max_rel_bound": float(np.max(bd / np.abs(ref))),
                      "max_rel_diff_vs_fp64": float(np.max(np.abs(v - v64) / np.abs(ref))),
                      "max_rel_err_vs_oracle": float(np.max(np.abs(v - ref) / np.abs(ref))),
                      "within_bound": bool(np.all(np.abs(v - v64) <= bd + 1e-13 * np.abs(ref)))})
    ok = [r for r in table if r["max_rel_bound"] <= 1e-10 and r["within_bound"]]
    chosen = min(ok, key=lambda r: r["ms_per_step"]) if ok else None
    return {"workload": "the ATM step above with EZ_PREC_MIXED: reciprocal terms with a >= a_mix at every node "
                        "of a 64-node wave block in FP32, the rest FP64; a-priori bound per result",
            "fp64": {"ms_per_step": round(ms_fp64, 5), "node_kernel_ms": round(node_ms_fp64, 5)},
            "table": table,
            "chosen": chosen,
            "speedup_step_vs_fp64": (ms_fp64 / chosen["ms_per_step"]) if chosen else None,
            "speedup_node_kernel_vs_fp64": (node_ms_fp64 / chosen["node_kernel_ms"]) if chosen else None,
            "equal_accuracy": "both within 1e-12 of the oracle on the identical plan; the mixed bound certifies "
                              "<= 1e-10 relative"}


def phase_leg(args) -> dict:
    """fcc / bcc phase diagram over (p, lam) for LJ (12,6) and (8,4) with ATM
    coupling lam (paper, Sec. 5) and the Bain path (bct, c/a from 0.9 to 1.6)."""
    import numpy as np
    import torch
    from paper_2504_11989_amd import phase
    import workloads as W
    spec = dict(W.SPEC_FULL_3D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    const = phase.lattice_constants(np.stack([W.A_FCC_NN1, W.A_BCC_NN1]), spec)
    torch.cuda.synchronize()
    t_const = time.perf_counter() - t0
    f = {k: v[0:1] for k, v in const.items()}
    b = {k: v[1:2] for k, v in const.items()}
    ps = np.linspace(0.0, 2.0, 32)
    lams = np.linspace(0.0, 4.0, 32)
    out = {"workload": "fcc and bcc (unit nearest-neighbour distance) at the full plan: Z_12, Z_6, Z_8, Z_4 "
                       "(two-body zeta functions) and E_ATM in one call; H minimised over R on a 32 x 32 "
                       "(p in [0,2], lam in [0,4]) grid for LJ (12,6) and (8,4); Bain path of 64 bct lattices",
           "constants_ms": round(1e3 * t_const, 3),
           "constants": {k: [float(x) for x in v] for k, v in const.items()}}
    t1 = time.perf_counter()
    for lj in ((12, 6), (8, 4)):
        dh = phase.phase_diagram(f, b, ps, lams, lj)
        lc = phase.critical_coupling(f, b, ps, lj, lam_max=20.0)
        out[f"lj_{lj[0]}_{lj[1]}"] = {
            "phase_map_rows_p_cols_lam": ["".join("b" if x < 0 else "f" for x in row) for row in dh],
            "lam_c_at_p": {f"{p:.3f}": float(l) for p, l in zip(ps[::8], lc[::8])},
            "lam_c_range": [float(np.nanmin(lc)), float(np.nanmax(lc))]}
    out["host_minimisation_s"] = round(time.perf_counter() - t1, 3)
    cas = np.linspace(0.9, 1.6, 64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    H0, s0, cb = phase.bain_path(cas, spec, (12, 6), 0.0, 0.0)
    torch.cuda.synchronize()
    lam_c0 = float(out["lj_12_6"]["lam_c_at_p"]["0.000"])
    H1, _ = phase.h_min(cb, (12, 6), 0.0, lam_c0)
    out["bain_path"] = {"c_over_a": [round(float(x), 5) for x in cas[::4]],
                        "H_min_lam0": [float(x) for x in H0[::4]],
                        "H_min_lam_c": [float(x) for x in H1[::4]],
                        "batched_call_ms": round(1e3 * (time.perf_counter() - t2), 3),
                        "argmin_c_over_a_lam0": float(cas[int(np.argmin(H0))]),
                        "argmin_c_over_a_lam_c": float(cas[int(np.argmin(H1))])}
    return out


def highn_leg(args) -> dict:
    """Ring sums zeta^(n)(3, ..., 3) on the square and hexagonal lattices for
    n = 2 .. 51 (paper, Sec. 4.4: the 100-dimensional sum at n = 51), their ratio to
    Z_3(0)^n and the time per sum against n; and the n_q study on A_kappa Z^2
    (Sec. 4.1) as one batched call with per-lattice plans."""
    import numpy as np
    import torch
    import paper_2504_11989_amd as ez
    from paper_2504_11989_amd import autotune
    import workloads as W
    spec = dict(W.SPEC_2D)
    out = {"workload": "zeta^(n)(3,...,3), n = 2..51, sq and hex, full 2D plan (n_q = 14, 96 graded u); "
                       "zeta^(3)(1,3,5) on A_kappa, kappa = 1, 2, 3, n_q = 4..20 in one call"}
    ns = [2, 3, 4, 6, 8, 12, 16, 24, 32, 40, 51]
    for name, A in (("sq", np.eye(2)), ("hex", W.A_HEX)):
        z0 = float(ez.epstein_zeta(A, [3.0], np.zeros((1, 2)), np.zeros((1, 2))).cpu().numpy()[0, 0].real)
        rows = []
        for n in ns:
            ez.nbody_lattice_sum(A, [3.0] * n, spec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                v = ez.nbody_lattice_sum(A, [3.0] * n, spec)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            zn = v.item()
            rows.append({"n": n, "zeta_n": zn, "zeta_n_over_Z0_n": zn / z0 ** n, "ms": round(ms, 4)})
        out[name] = {"Z3_0": float(z0), "rows": rows}
    kappas = [1.0, 2.0, 3.0]
    nqs = list(range(4, 21, 2))
    A = np.stack([W.a_kappa(k) for k in kappas for _ in nqs])
    specs = [dict(spec, n_q=q) for _ in kappas for q in nqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = ez.lattice_sums(A, [1.0, 3.0, 5.0], [(0, 1.0, [(0, 1), (1, 1), (2, 1)])], 1, specs).cpu().numpy()[:, 0]
    t_batch = time.perf_counter() - t0
    got = got.reshape(len(kappas), len(nqs))
    study = []
    for i, k in enumerate(kappas):
        ref = got[i, -1]
        err = [float(min(abs(x - ref), abs(x - ref) / abs(ref))) for x in got[i, :-1]]
        e = np.array(err)
        m = e > 1e-13
        rho_fit = float(np.exp(-np.polyfit(np.array(nqs[:-1])[m], np.log(e[m]), 1)[0] / 2.0)) if m.sum() >= 3 else None
        study.append({"kappa": k, "n_q": nqs[:-1], "E": err, "rho_fit": rho_fit,
                      "rho_bound": autotune.rho_bound(W.a_kappa(k)),
                      "n_q_for_1e-12": autotune.nq_for(W.a_kappa(k), 1e-12)})
    out["kappa_study"] = {"batched_call_s": round(t_batch, 4), "rows": study}
    return out


def meromorphic_leg(args) -> dict:
    """The one-dimensional three-body zeta function zeta^(3)_Z(nu, nu, nu) along
    -2 <= nu <= 3 in steps of 1/20 with the offset 1/50 (paper, Sec. 4.3, the scan of
    the meromorphic continuation): 101 sums with non-integer exponents, GPU time
    per sum and the largest deviation from the oracle on every 10th point."""
    import numpy as np
    import torch
    import oracle
    import paper_2504_11989_amd as ez
    import workloads as W
    spec = dict(W.SPEC_1D)
    nus = [-2.0 + j / 20.0 + 1.0 / 50.0 for j in range(101)]
    vals = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for nu in nus:
        vals.append(ez.nbody_lattice_sum(np.eye(1), [nu] * 3, spec))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    vals = [v.item() for v in vals]
    # relative deviation, and the deviation over the parity bar max(1e-12 |v|, 4e-15 (|H| + |N|))
    # that allows for the cancellation of the Hadamard and node parts near the poles
    err, over = 0.0, 0.0
    for j in range(0, 101, 10):
        ref, parts = oracle.nbody(np.eye(1), [nus[j]] * 3, spec, parts=True)
        dev = abs(vals[j] - ref)
        err = max(err, dev / max(abs(ref), 1e-300))
        over = max(over, dev / max(1e-12 * abs(ref), 4e-15 * float(np.abs(parts).sum())))
    return {"workload": "zeta^(3)_Z(nu,nu,nu), nu = -2 + j/20 + 1/50, j = 0..100, 1-D plan (1024 graded u-nodes)",
            "sums": len(nus), "ms_per_sum": round(1e3 * dt / len(nus), 4),
            "nu": [round(x, 4) for x in nus[::10]], "values": [vals[j] for j in range(0, 101, 10)],
            "max_rel_err_vs_oracle_every_10th": err, "max_deviation_over_parity_bar": over}


def batch_scan_leg(args) -> dict:
    """The node stage of the three-lattice ATM call at several copies of the batch
    (sc, fcc, bcc repeated), HIP events on the launch stream, 10 calls each: how far
    the three-lattice call is from the device's throughput at large batches."""
    import numpy as np
    import torch
    import paper_2504_11989_amd as ez
    import workloads as W
    from paper_2504_11989_amd import _native as nat
    spec = dict(W.SPEC_FULL_3D)
    lats = [W.sc(), W.fcc(), W.bcc()]
    rows = []
    for r in (1, 2, 4, 8, 16):
        A = torch.tensor(np.stack(lats * r), dtype=torch.float64, device="cuda")
        ez.atm_energy(A, spec)
        torch.cuda.synchronize()
        nat.timing_reset()
        nat.timing_enable(True)
        for _ in range(10):
            ez.atm_energy(A, spec)
        torch.cuda.synchronize()
        nat.timing_enable(False)
        ms, n = nat.timing_read(nat.KERNEL_NODES)
        mt, _ = nat.timing_read(nat.KERNEL_NODES_TAIL)
        per_call = (ms + mt) / 10
        flops = node_kernel_flops_per_node(spec["lam"], spec["a_cut"], 4) * W.n_nodes(3, spec) * 3 * r
        rows.append({"lattices": 3 * r, "node_ms_per_call": round(per_call, 4),
                     "ms_per_lattice": round(per_call / (3 * r), 5),
                     "frac_fp64_peak": round(flops / (per_call * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS, 4)})
    return {"workload": "three-lattice ATM call (full plan) repeated 1, 2, 4, 8, 16 times in one batch",
            "rows": rows}


def direct_leg(args) -> dict:
    """GPU direct sums of the ATM energy over boxes (ez_direct_atm): the paper's
    printed direct sums (Lambda = Z at L = 5000, the square lattice at L = 250 and its
    high-precision reference at L = 1600), the L^-4 Richardson extrapolation of the
    square-lattice box sums against the Epstein zeta method on the full 2-D plan."""
    import json as _json
    import numpy as np
    import torch
    import paper_2504_11989_amd as ez
    import workloads as W
    paper = _json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    out = {"workload": "E_L = (1/6) sum over x, y in A{-L..L}^d of U_ATM(0, x, y); square lattice with the orbit "
                       "reduction of the signed coordinate permutations"}
    rows = []
    for name, A, L, sym, key in (("Z", np.eye(1), 5000, False, "atm_1d_direct_L5000"),
                                 ("sq", np.eye(2), 250, True, "atm_2d_sq_direct_L250"),
                                 ("sq", np.eye(2), 1600, True, "atm_2d_sq_reference_L1600")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v = ez.direct_atm(A, L, symmetry=sym)
        dt = time.perf_counter() - t0
        d = A.shape[0]
        n = (2 * L + 1) ** d
        p = paper[key]["value"]
        # pairs: ordered pairs of the full box; terms_per_s: terms the kernel evaluates per
        # second (about pairs / 8 under the orbit reduction of the square lattice)
        rows.append({"lattice": name, "L": L, "value": v, "paper": p, "rel_diff_vs_paper": abs(v - p) / abs(p),
                     "seconds": round(dt, 3), "pairs": float(n) * float(n - 2),
                     "terms_per_s": float(n) * float(n - 2) / dt / (8.0 if sym and d == 2 else 1.0)})
    out["sums"] = rows
    e = ez.atm_energy(np.eye(2)[None], W.SPEC_2D).item()
    v2, v4 = ez.direct_atm(np.eye(2), 200, symmetry=True), ez.direct_atm(np.eye(2), 400, symmetry=True)
    ext = (16.0 * v4 - v2) / 15.0
    out["square_epstein"] = e
    out["square_richardson_L200_L400"] = ext
    out["rel_diff_epstein_vs_richardson"] = abs(e - ext) / abs(ext)
    return out


def c5_leg(args) -> dict:
    """Differentiation and n-body sums.  (1) dH/dA of H = E_LJ(12-6) + c E_ATM + p V
    from the adjoint kernels against central differences of the GPU value (h =
    1e-6) on 16 generator matrices perturbed by up to 10% from fcc/bcc (seed 5),
    c = 1, p = 0.5.  (2) The (c, p) scan: c in linspace(0, 2, 32), p in
    linspace(0, 1, 32), BFGS from a perturbed fcc and a perturbed bcc start at
    every point, all 2048 minimisations batched (one lattice-sum call with
    derivatives per trial step); the winning lattice per point classified by its
    neighbour shells.  (3) Ring sums zeta^(n)(6, ..., 6), n = 2..6, on the simple
    cubic lattice, full plan."""
    import numpy as np
    import torch

    import oracle
    import workloads as W
    import paper_2504_11989_amd as ez
    from paper_2504_11989_amd import enthalpy as H

    spec = dict(W.SPEC_SMALL_3D)
    out = {"workload": "H = E_LJ(12-6) + c E_ATM + p V per particle, 3x3 generator matrices; "
                       "(c, p) grid 32 x 32, c in [0,2], p in [0,1]: fcc vs bcc minimised over the scale, "
                       "then general-matrix minimisation from the winners perturbed by up to 10% (seed 5); ring sums zeta^(n)(6,...,6) n = 2..6 on sc; FP64",
           "plan": spec}
    # (1) gradient check, batched over the 16 matrices
    A = W.c5_perturbed(count=16)
    c, p = 1.0, 0.5
    At = torch.tensor(A, device="cuda")
    _, g, _, _ = H.enthalpy(At, c, p, spec)
    g = g.cpu().numpy()
    hh = 1e-6
    fd = np.zeros_like(g)
    for i in range(3):
        for j in range(3):
            Ap, Am = A.copy(), A.copy()
            Ap[:, i, j] += hh
            Am[:, i, j] -= hh
            hp = H.enthalpy(torch.tensor(Ap, device="cuda"), c, p, spec)[0].cpu().numpy()
            hm = H.enthalpy(torch.tensor(Am, device="cuda"), c, p, spec)[0].cpu().numpy()
            fd[:, i, j] = (hp - hm) / (2 * hh)
    err = max(float(np.linalg.norm(g[b] - fd[b]) / np.linalg.norm(fd[b])) for b in range(len(A)))
    out["grad_check"] = {"matrices": len(A), "c": c, "p": p, "h": hh, "max_rel_err_adjoint_vs_central_fd": err}
    # (2) the phase scan: Bain-path minimisation from bcc and fcc starts, then the
    # general-matrix minimisation from every perturbed winner
    cs, ps = W.c5_grid(32)
    n_eval = {"calls": 0, "lattices": 0}
    inner = H.enthalpy

    def counted(At, *a, **k):
        n_eval["calls"] += 1
        n_eval["lattices"] += int(At.shape[0])
        return inner(At, *a, **k)

    H.enthalpy = counted
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = H.phase_scan(cs, ps, spec, max_iter=args.c5_iters, stability=True, stability_iter=100,
                           stability_stride=4, verbose=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        H.enthalpy = inner
    phase = res["phase"]
    gen = res["general"]
    nmin = res["H"].size + gen.size
    names, counts = np.unique(phase.astype(str), return_counts=True)
    gnames, gcounts = np.unique(gen.astype(str), return_counts=True)
    out["scan"] = {"grid": [len(cs), len(ps)], "minimisations": int(nmin), "seconds": dt,
                   "minimisations_per_s": nmin / dt,
                   "fcc_vs_bcc": {"form": "H minimised over the lattice scale R of fcc and of bcc (paper, Sec. 5)",
                                  "problems": int(res["H"].size), "iterations": int(res["iterations"]),
                                  "converged": int(res["converged"].sum()),
                                  "phase_counts": {str(k): int(v) for k, v in zip(names, counts)},
                                  "phase_map_rows_c_cols_p": ["".join(str(x)[0] for x in row) for row in phase],
                                  "H_fcc_c0_p0": float(res["H"][0, 0, 0])},
                   "general_matrix": {"form": "H minimised over all 9 entries from the winner perturbed by up to 10%, "
                                              "every 4th point in c and p (8 x 8)",
                                      "problems": int(gen.size), "iterations": int(res["general_iterations"]),
                                      "converged": int(res["general_converged"].sum()),
                                      "degenerate": int(res["general_degenerate"].sum()),
                                      "outcome_counts": {str(k): int(v) for k, v in zip(gnames, gcounts)},
                                      "outcome_map_rows_c_cols_p": ["".join(str(x)[0] for x in row) for row in gen]},
                   "batched_evaluations": n_eval["calls"],
                   "lattice_evals_with_grad_per_s": n_eval["lattices"] / dt}
    # (3) ring sums on sc, full plan, timed; the small plan against the oracle
    full = dict(W.SPEC_FULL_3D)
    ring = {}
    for n in range(2, 7):
        v = ez.nbody_lattice_sum(W.sc(), [6.0] * n, full)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            v = ez.nbody_lattice_sum(W.sc(), [6.0] * n, full)
        torch.cuda.synchronize()
        vs = ez.nbody_lattice_sum(W.sc(), [6.0] * n, spec).item()
        ref = oracle.nbody(W.sc(), [6.0] * n, spec)
        ring[str(n)] = {"value_full_plan": v.item(), "ms": 1e3 * (time.perf_counter() - t0) / 5,
                        "rel_err_vs_oracle_small_plan": abs(vs - ref) / abs(ref)}
    out["ring_sums_sc_nu6"] = ring
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched 4096-lattice scan leg")
    ap.add_argument("--c3-reps", type=int, default=3)
    ap.add_argument("--no-c4", action="store_true", help="skip the mixed-precision Epstein grid leg")
    ap.add_argument("--c4-reps", type=int, default=3)
    ap.add_argument("--no-c5", action="store_true", help="skip the enthalpy scan and ring-sum leg")
    ap.add_argument("--c5-iters", type=int, default=100)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision ATM leg")
    ap.add_argument("--no-phase", action="store_true", help="skip the phase-diagram / Bain-path leg")
    ap.add_argument("--no-highn", action="store_true", help="skip the high-n / kappa-study leg")
    ap.add_argument("--no-direct", action="store_true", help="skip the GPU direct-sum leg")
    ap.add_argument("--batch-scan", action="store_true",
                    help="also time the node stage of the ATM call at 1-16 copies of the three lattices")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 1 GiB device-to-device copies (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the lattice sums shard trivially "
              "by lattice or node tile; no multi-GPU path is built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 27                     # 2^27 doubles = 1 GiB
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": n * 8, "copies": 3}), flush=True)
        return 0

    import paper_2504_11989_amd as ez
    from paper_2504_11989_amd import _native as nat
    import workloads as W

    dev = torch.device("cuda:0")
    spec = dict(W.SPEC_FULL_3D)
    names = ["sc", "fcc", "bcc"]
    A = torch.tensor(np.stack([W.c2_lattices()[n] for n in names]), dtype=torch.float64, device=dev)
    nodes = W.n_nodes(3, spec)
    n_nu = 4

    out = ez.atm_energy(A, spec)
    for _ in range(args.warmup):
        out = ez.atm_energy(A, spec)
    torch.cuda.synchronize()

    # accuracy against the oracle on the identical plan (stored by tests/golden/make_oracle_golden.py)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_c2_full.json")))
    got = out.cpu().numpy()
    max_rel = max(abs(got[i] - gold["atm"][n]) / abs(gold["atm"][n]) for i, n in enumerate(names))

    # timed region: K steps, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ez.atm_energy(A, spec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps

    # per-kernel times: HIP events recorded by the library on the launch stream
    nat.timing_reset()
    nat.timing_enable(True)
    for _ in range(min(args.steps, 50)):
        ez.atm_energy(A, spec)
    torch.cuda.synchronize()
    nat.timing_enable(False)
    kt = {k: nat.timing_read(i) for k, i in [("setup", nat.KERNEL_SETUP), ("nodes", nat.KERNEL_NODES),
                                              ("nodes_tail", nat.KERNEL_NODES_TAIL),
                                              ("taylor", nat.KERNEL_TAYLOR),
                                              ("hadamard", nat.KERNEL_HADAMARD),
                                              ("finalize", nat.KERNEL_FINALIZE)]}

    # the same workload with dE/dA (adjoint kernels), timed the same way
    adj = None
    if not args.no_adjoint:
        for _ in range(max(1, args.warmup // 2)):
            ez.atm_energy(A, spec, grad=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        n_adj = max(1, args.steps // 2)
        for _ in range(n_adj):
            Eg, gA = ez.atm_energy(A, spec, grad=True)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        # adjoint node kernel time with the timing hooks, in calls of their own
        nat.timing_reset()
        nat.timing_enable(True)
        for _ in range(min(n_adj, 20)):
            ez.atm_energy(A, spec, grad=True)
        torch.cuda.synchronize()
        nat.timing_enable(False)
        na = nat.timing_read(nat.KERNEL_NODES_ADJ)
        eg = Eg.cpu().numpy()
        adj = {"unit": "ATM lattice sums with dE/dA per s", "value": len(names) * n_adj / (tb - ta),
               "ms_per_step": 1e3 * (tb - ta) / n_adj,
               "node_adj_kernel_ms": round(na[0] / max(1, na[1]), 5),
               "max_rel_err_vs_oracle": max(abs(eg[i] - gold["atm"][n]) / abs(gold["atm"][n])
                                            for i, n in enumerate(names)),
               "homogeneity_residual": float(max(abs(np.trace(A[i].cpu().numpy().T @ gA[i].cpu().numpy())
                                                     + 9.0 * eg[i]) / abs(9.0 * eg[i]) for i in range(len(names))))}
    sums_per_s = len(names) * args.steps / elapsed
    evals_per_s = len(names) * nodes * n_nu * args.steps / elapsed

    # node stage: the tile kernel plus, when the tile count passes a multiple of a
    # round of workgroups by a little, the split kernel that takes the last tiles
    node_ms = kt["nodes"][0] / max(1, kt["nodes"][1]) + kt["nodes_tail"][0] / max(1, kt["nodes"][1])
    flops_launch = node_kernel_flops_per_node(spec["lam"], spec["a_cut"], n_nu) * nodes * len(names)
    achieved = flops_launch / (node_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_sha") == kernel_source_sha():
            traffic = tr["bytes_per_launch"]
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP64_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 5), "traffic": traffic,
                "kernel": "ez_node_kernel<3,4,1>" + (" + ez_node_split_kernel<3,4,1> (last tiles)"
                                                     if kt["nodes_tail"][1] else ""),
                "kernel_ms": round(node_ms, 5),
                "flops_per_launch": flops_launch}

    line = {
        "metric": METRIC,
        "value": sums_per_s,
        "unit": "ATM lattice sums/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "d=3 ATM cohesive energy per particle, sc/fcc/bcc at unit density, "
                               "263424 nodes per lattice (12 Duffy blocks x 14^2 v x 112 graded u) + Hadamard part, FP64",
                   "lattices": len(names), "nodes_per_lattice": nodes, "spec": spec},
        "epstein_evals_per_s": evals_per_s,
        "max_rel_err_vs_oracle": max_rel,
        "kernel_ms": {k: round(v[0] / max(1, v[1]), 5) for k, v in kt.items()},
        "roofline": roofline,
        "adjoint": adj,
        "c3_scan": None,
        "c4_grid": None,
        "c5": None,
        "mixed": None,
        "phase": None,
        "highn": None,
        "meromorphic_1d": None,
        "direct_sums": None,
        "cpu_baseline": None,
    }
    def leg(name, fn):
        print(f"bench: {name} ...", file=sys.stderr, flush=True)
        t = time.perf_counter()
        r = fn()
        print(f"bench: {name} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
        return r

    if not args.no_mixed:
        line["mixed"] = leg("mixed precision", lambda: mixed_leg(args, A, spec, gold, names, ms_step, node_ms))
    if not args.no_phase:
        line["phase"] = leg("phase diagram", lambda: phase_leg(args))
    if not args.no_highn:
        line["highn"] = leg("high-n sums", lambda: highn_leg(args))
        line["meromorphic_1d"] = leg("1-D continuation scan", lambda: meromorphic_leg(args))
    if not args.no_direct:
        line["direct_sums"] = leg("direct sums", lambda: direct_leg(args))
    if args.batch_scan:
        line["c2_batch_scan"] = leg("batch scan", lambda: batch_scan_leg(args))
    if not args.no_c3:
        line["c3_scan"] = leg("c3 scan", lambda: c3_scan_leg(args))
    if not args.no_c4:
        line["c4_grid"] = leg("c4 grid", lambda: c4_grid_leg(args))
    if not args.no_c5:
        line["c5"] = leg("c5 enthalpy", lambda: c5_leg(args))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = leg("cpu baseline", lambda: cpu_baseline(spec))
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

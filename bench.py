#!/usr/bin/env python3
"""Benchmark of the SHMM hot path on one MI355X.

One step = one pass of the hot path over the four-level cellular workload
(psi = sum_{k=1,4,16,64} k^(-4/3) sin(kx+p1) sin(ky+p2), kappa = 1e-2, 4 levels
of 64 patches of 128^2 cells) plus the shear check instance v = (0, sin 16x):
band filter, top-down Algorithm 2, then every phase (base, step plan, local
solves, FP64 effective diffusivity, level combination), all on the GPU with
the inputs resident in HBM.

Prints one JSON line on stdout; progress goes to stderr.
"""
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

METRIC = "κ_eff estimates/s + Gpoint-steps/s; surrogate vs plain at ≤1% κ_eff error"
# Algorithmic FP32 work of one point-step (one cell of one patch, one classic
# RK4 step, both correctors): per corrector 4 evaluations of the 9-point
# operator with forcing (6 FMA + 4 ADD = 16 flop), 3 stage inputs (2 flop each)
# and the final update (8 flop): 78 flop; two correctors.
FLOP_PER_POINT_STEP = 156
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak (256 CU, 2.4 GHz)
# HBM bytes per full-phase launch of k_solve_resident_e<128, 32, 8> on this
# workload, from rocprofv3 FETCH_SIZE (x2.0) and WRITE_SIZE (x1.0), the scale
# factors read off a 1 GiB device copy.  Valid only for the kernel code they
# were taken on (first 16 hex digits of the SHA-256 of solve.hip without its
# comments and blank lines); otherwise reported null.
SOLVE_TRAFFIC = {"code_sha256": "20887aa200990312", "variant": 5,
                 "bytes_per_launch": (2 * 12634.9 + 8832.0) * 1024}
SOLVE_KERNELS_128 = {0: "k_solve_resident<128,32>", 1: "k_solve_rows<128,2,16>", 2: "k_solve_rows<128,2,8>",
                     3: "k_solve_resident_e<128,32>", 4: "k_solve_resident_e<128,16>",
                     5: "k_solve_resident_e<128,32,8>", 6: "k_solve_resident_e<128,32,16>"}


def solve_traffic():
    """The counted HBM bytes of one solve launch while the code of the solve
    kernels (solve.hip and its stage header, comments aside) is the code the
    counters were taken on; None otherwise."""
    import hashlib
    lines = []
    for f in ("solve.hip", "solve_stage.h"):
        lines += open(os.path.join(ROOT, "paper_1510_00451_amd", "csrc", f)).read().split("\n")
    code = "\n".join(l.split("//")[0].rstrip() for l in lines if l.split("//")[0].strip())
    h = hashlib.sha256(code.encode()).hexdigest()[:16]
    return SOLVE_TRAFFIC["bytes_per_launch"] if h == SOLVE_TRAFFIC["code_sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    import flowgen
    main = flowgen.config_four_level_cellular(seed=0, n=128, lattice=8)
    shear = flowgen.config_shear(k=16, V=1.0, kappa=1e-2, n=128, levels=2, thresh=[8])
    return [main, shear]


def cpu_baseline(steps_sample: int = 10000, domains_sample: int = 32):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    the finest-level patches of the four-level instance, a fixed number of RK4
    steps each, OpenMP over (patch, corrector)."""
    import oracle
    import flowgen
    p = flowgen.config_four_level_cellular(seed=0, n=128, lattice=8)
    doms = [d for d in oracle.domain_table(p) if d.level == 3][:domains_sample]
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    fields = [oracle.level_fields(p, lv, pt, d) for d in doms]
    vx = np.concatenate([f[1].ravel() for f in fields])
    vy = np.concatenate([f[2].ravel() for f in fields])
    f1 = np.concatenate([f[3].ravel() for f in fields])
    f2 = np.concatenate([f[4].ravel() for f in fields])
    Kb = np.tile([p.kappa, 0.0, p.kappa], (len(doms), 1))
    vmax = max(oracle.advection_bound(f[1], f[2]) for f in fields)
    dt, _ = oracle.plan_steps(128, doms[0].h, Kb[0], vmax, p.dt_frac, p.delta)
    t0 = time.perf_counter()
    oracle.local_solve_batch([d.n for d in doms], [d.h for d in doms], vx, vy, f1, f2, Kb,
                             [dt] * len(doms), [steps_sample] * len(doms))
    el = time.perf_counter() - t0
    pts = sum(d.n * d.n for d in doms) * steps_sample
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pts / el / 1e9, "unit": "Gpoint-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(doms)} finest-level 128^2 patches x {steps_sample} RK4 steps "
                      f"(both correctors, FP64), {el:.1f} s"}


def surrogate_leg(flows_train: int, flows_eval: int, steps: int = 1500, members: int = 4, lattice: int = 16):
    """Learned surrogate against the plain local solve.

    Labels: plain-path solves of the finest-level patches of flows from the
    uneven-batch generator (seeds 100000+, n = 128, 16 x 16 patches, isotropic
    base).  Training: the rescaling symmetry (two extra copies), an ensemble of
    `members` networks, Adam at batch 4096 on gradients clipped to norm 1.
    Members that failed to train are dropped and the gate (spread threshold,
    enhancement limit) is calibrated on a held-out tenth of the labels.  Evaluation: finest-level patches of
    continuous-spectrum flows (seeds 200000+), timed in both forms from the band
    filter on, with the inputs resident."""
    import torch
    import flowgen
    from paper_1510_00451_amd import abi
    from paper_1510_00451_amd import surrogate as GS
    t0 = time.perf_counter()
    per = max(1, 1024 // (lattice * lattice))          # about 1024 finest patches per batch
    batches = ([flowgen.config_batched_instance(100000 + i + j, n=128, lattice=lattice)
                for j in range(min(per, flows_train - i))] for i in range(0, flows_train, per))
    data = GS.labelled_set(batches, log=log, adaptive=True)
    t_label = time.perf_counter() - t0
    held, train = GS.split(data, 0.1, seed=0)
    rng = np.random.default_rng(1)
    train = GS.Dataset.concat([train] + [train.rescaled(rng.uniform(-1.5, 1.5, train.x.shape[0]))
                                         for _ in range(2)])
    ctx = abi.Context(0)
    mu = train.x.double().mean(0).cpu().numpy()
    sg = train.x.double().std(0).cpu().numpy() + 1e-6
    ens = GS.Ensemble(ctx, members, mu, sg, seed0=11)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = GS.train(ens, train, steps=steps, batch=4096, lr0=1e-3, seed=5, log=log, clip=1.0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    member_losses = ens.prune(held)
    log(f"surrogate: held-out member losses {member_losses}, {ens.E} kept")
    lo, hi = GS.gate_range(train, 0.1)
    tau, emax, held_acc = GS.calibrate_gate(ens, held, lo, hi)
    log(f"surrogate: {data.x.shape[0]} labels in {t_label:.1f} s, trained in {t_train:.1f} s, "
        f"tau {tau}, emax {emax}, held-out accepted {held_acc:.3f}")

    # all evaluation flows in one phase: the fallback solves of every flagged
    # patch then share one launch, as they would in a stream of patches
    ph = GS.IsotropicPhase([flowgen.config_continuous(seed=200000 + i) for i in range(flows_eval)])
    torch.cuda.synchronize()
    a = time.perf_counter()
    ph.prepare()
    Kp = ph.plain()
    torch.cuda.synchronize()
    b = time.perf_counter()
    ph.prepare()
    Ks = ph.surrogate(ens, lo, hi, tau, emax)
    torch.cuda.synchronize()
    c = time.perf_counter()
    t_plain, t_surr = b - a, c - b
    act = ph.active
    n_est = int(act.sum())
    Kp_h, Ks_h = Kp.cpu().numpy().copy(), Ks.cpu().numpy().copy()
    errs = [GS.relative_frobenius(Ks_h[act], Kp_h[act])]
    flagged = [ph.flags.cpu().numpy()[act].astype(bool)]
    # both forms again with the quasi-stationary stop (plain solves and fallback)
    ph.prepare()
    planned_steps = ph.point_steps
    torch.cuda.synchronize()
    a = time.perf_counter()
    ph.prepare()
    Kpa = ph.plain(adaptive=True)
    torch.cuda.synchronize()
    b = time.perf_counter()
    tab = ph.H.ctx.shmm_ctx_table()[0][ph.first:ph.first + ph.count]
    taken = int(np.sum(tab["n"].astype(np.int64) ** 2 * tab["nsteps"].astype(np.int64)))
    Kpa_h = Kpa.cpu().numpy().copy()
    ph.prepare()
    Ksa = ph.surrogate(ens, lo, hi, tau, emax, adaptive=True)
    torch.cuda.synchronize()
    c = time.perf_counter()
    t_plain_a, t_surr_a = b - a, c - b
    err_a = GS.relative_frobenius(Ksa.cpu().numpy()[act], Kp_h[act])
    ph.close()
    err = np.concatenate(errs)
    fl = np.concatenate(flagged)
    ctx.close()
    return {
        "estimates_per_s": round(n_est / t_surr, 1),
        "plain_estimates_per_s": round(n_est / t_plain, 1),
        "speedup": round(t_plain / t_surr, 2),
        "err_vs_plain": {"mean": float(err.mean()), "p99": float(np.quantile(err, 0.99)),
                         "max": float(err.max()), "frac_over_1pct": float(np.mean(err > 0.01))},
        "fallback_frac": float(fl.mean()),
        "adaptive": {"estimates_per_s": round(n_est / t_surr_a, 1),
                     "plain_estimates_per_s": round(n_est / t_plain_a, 1),
                     "speedup": round(t_plain_a / t_surr_a, 2),
                     "plain_steps_taken_fraction": round(taken / planned_steps, 4),
                     "plain_max_rel_K_vs_planned": float(np.max(GS.relative_frobenius(Kpa_h[act], Kp_h[act]))),
                     "err_vs_planned_plain": {"mean": float(err_a.mean()), "p99": float(np.quantile(err_a, 0.99)),
                                              "max": float(err_a.max())}},
        "tau": tau, "emax": emax if math.isfinite(emax) else None, "held_out_accepted": round(held_acc, 4),
        "eval": f"{flows_eval} continuous-spectrum flows (kappa 1e-3, 1<=|k|<=512, |psi_k|~|k|^-7/3) x "
                f"256 finest-level 128^2 patches, isotropic base; {n_est} estimates",
        "train": {"labels": int(data.x.shape[0]), "flows": flows_train, "patches_per_flow": lattice * lattice,
                  "label_s": round(t_label, 1),
                  "train_s": round(t_train, 2), "steps": steps, "batch": 4096, "clip": 1.0, "members": members,
                  "members_kept": ens.E, "held_out_member_losses": [round(float(v), 6) for v in member_losses],
                  "final_loss": hist[-1] if hist else None},
    }


def continuous_leg(adaptive: bool = True):
    """One full pass over the five-level continuous-spectrum flow (256 patches
    of 128^2 per level): a second throughput figure at full occupancy; then
    (adaptive) the same pass with the quasi-stationary stop: its estimates/s,
    the fraction of the planned point-steps taken and the largest relative
    change of the final K."""
    import torch
    import flowgen
    from paper_1510_00451_amd.hierarchy import Hierarchy
    H = Hierarchy([flowgen.config_continuous(seed=0)], keep_psi=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = H.result()
    out = {"workload": "continuous-5level-256x128 (kappa 1e-3, 1<=|k|<=512)",
           "gpoint_steps_per_s": round(res.point_steps / el / 1e9, 3),
           "kappa_eff_estimates_per_s": round(len(res.R) / el, 2), "pass_s": round(el, 3)}
    if adaptive:
        t0 = time.perf_counter()
        H.run(adaptive=True)
        torch.cuda.synchronize()
        ela = time.perf_counter() - t0
        ra = H.result()
        d = np.abs(ra.K_total - res.K_total).max() / np.abs(res.K_total).max()
        out["adaptive"] = {"kappa_eff_estimates_per_s": round(len(ra.R) / ela, 2), "pass_s": round(ela, 3),
                           "steps_taken_fraction": round(ra.point_steps / res.point_steps, 4),
                           "max_rel_K_vs_planned": float(d)}
    H.close()
    return out


def uneven_leg(instances: int, window: int):
    """The uneven batch (generator seeds 0.., kappa, levels, slope and patch size
    drawn per instance; 4 x 4 patches per level, n from 32 to 256 mixed in
    every phase): one pass with every local solve capped at `window` steps,
    after tuning the kernels on the first phase."""
    import torch
    import flowgen
    from paper_1510_00451_amd.hierarchy import Hierarchy
    from paper_1510_00451_amd import autotune
    H = Hierarchy([flowgen.config_batched_instance(s) for s in range(instances)], keep_psi=False)
    H.run(steps=1)
    torch.cuda.synchronize()
    tuned = autotune.tune_solve(H, phase=0, steps=50, repeats=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.run(steps=window)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    table = H.ctx.shmm_ctx_table()[0]
    ns = np.minimum(table["nsteps"].astype(np.int64), window)
    pts = int(np.sum(table["n"].astype(np.int64) ** 2 * ns))
    sizes = {int(n): int(np.sum(table["n"] == n)) for n in sorted(set(table["n"].tolist()))}
    full = int(np.sum(table["n"].astype(np.int64) ** 2 * table["nsteps"].astype(np.int64)))
    H.close()
    return {"workload": f"uneven batch, {instances} instances (seeds 0-{instances - 1}), every solve capped "
                        f"at {window} steps",
            "gpoint_steps_per_s": round(pts / el / 1e9, 3), "window_s": round(el, 3),
            "domains_by_n": sizes, "autotune": {str(k): v["variant"] for k, v in tuned.items()},
            "full_run_point_steps_planned": full}


def _macro_dt(vx, vy, K, N, dt_frac, T):
    """RK4 step for the macro grid: dt_frac of the stability bound of the
    diffusion (4 K11 + 4 K22 + 2 |K12|) / h^2 and of the advection (Gershgorin
    bound of the face velocities) / h, rounded so the steps end at T."""
    h = 2.0 * math.pi / N
    rho = (4.0 * K[0] + 4.0 * K[2] + 2.0 * abs(K[1])) / h ** 2 / 2.785
    if vx is not None:
        ax, ay = np.abs(vx.reshape(N, N)), np.abs(vy.reshape(N, N))
        vmax = 0.5 * float(np.max(ax + np.roll(ax, -1, axis=1) + ay + np.roll(ay, -1, axis=0)))
        rho += vmax / h / 2.828
    steps = max(1, int(math.ceil(T / (dt_frac / rho))))
    return T / steps, steps


def oversampling_leg(seeds=(7, 8, 9), bands=((12, 20), (8, 16)), kappa: float = 0.1):
    """Oversampled patches against plain ones on scale-separated flows (random
    phases, |psi_k| ~ |k|^-2 on an annulus of wavenumbers, 256^2 grid).  The
    reference is the direct cell problem: one 256^2 patch covering the
    periodic domain.  Compared: 4 x 4 tiles of 64^2 (patch side H = pi / 2,
    the lattice spacing), patches of side 2H (128^2) averaged over the whole
    patch, the same averaged over the centred 64^2 window only, and the same
    again with the stream function tapered over 16 nodes at the patch edges
    (windowed patches), and with zero-frame (non-periodic) local problems.
    Reported:
    the relative Frobenius error of the patches' mean K against the direct K,
    and the median error of a single patch."""
    import flowgen
    from paper_1510_00451_amd.hierarchy import Hierarchy

    def rel(a, b):
        d = a - b
        return float(np.sqrt((d[0] ** 2 + 2 * d[1] ** 2 + d[2] ** 2) / (b[0] ** 2 + 2 * b[1] ** 2 + b[2] ** 2)))

    cases = []
    for seed in seeds:
        for k_lo, k_hi in bands:
            H = Hierarchy([flowgen.config_band_pass(seed, k_lo, k_hi, kappa, 256, 1, 256)])
            H.run()
            Kd = H.result().K_total[0]
            H.close()
            row = {"seed": seed, "band": [k_lo, k_hi], "K_direct": [round(float(x), 6) for x in Kd]}
            for name, n, inner, taper, frame in (("tiles_64", 64, 0, 0, 0), ("side_2H_whole", 128, 0, 0, 0),
                                                 ("side_2H_window_64", 128, 64, 0, 0),
                                                 ("side_2H_taper_16_window_64", 128, 64, 16, 0),
                                                 ("side_2H_zero_frame_window_64", 128, 64, 0, 1)):
                H = Hierarchy([flowgen.config_band_pass(seed, k_lo, k_hi, kappa, n, 4, 256)], keep_psi=taper > 0)
                H.estimator_inner = inner
                H.patch_taper = taper
                H.ctx.shmm_ctx_set_local_bc(frame)
                H.run()
                K = H.result().K_total
                H.close()
                row[name] = {"mean_err": round(rel(K.mean(0), Kd), 5),
                             "median_patch_err": round(float(np.median([rel(k, Kd) for k in K])), 4)}
            cases.append(row)
            log(f"oversampling seed {seed} band {k_lo}-{k_hi}: " +
                ", ".join(f"{k} {row[k]['mean_err']}" for k in ("tiles_64", "side_2H_whole", "side_2H_window_64",
                                                                 "side_2H_taper_16_window_64",
                                                                 "side_2H_zero_frame_window_64")))
    return {"workload": f"band-pass flows on a 256^2 grid, kappa {kappa}, 4 x 4 patch centres", "cases": cases}


def paper_tests_leg(n_k: int = 128, n_dns: int = 512):
    """The cellular examples of Section 4 (Tests 2 and 3), as printed and with
    the velocity scaled by 2 pi.  K: two-level SHMM (decomposition factor 5)
    against the direct cell problem of the full flow, on the wavenumbers
    divided by 5 (the same homogenized K) at n_k^2.  u: the Section 4
    problem (step data, u = 1 on x = 0 and 0 on x = 2 pi, y periodic) at
    t = 0.02 and t = 0.1 of the paper (x 4 pi^2 here): a direct simulation with the full
    velocity on n_dns^2 (FP32), against the homogenized equation with the
    SHMM K and with kappa alone (FP64, n_dns / 4), compared with the DNS
    averaged over y and over 4-cell blocks in x."""
    import torch
    import flowgen
    from paper_1510_00451_amd import abi
    from paper_1510_00451_amd.hierarchy import Hierarchy
    T = 0.4 * math.pi ** 2
    s = torch.cuda.current_stream().cuda_stream
    out = []
    for test in (2, 3):
        for label, scale in (("as printed", 1.0), ("velocity x 2 pi", 2.0 * math.pi)):
            rec = {"test": test, "scale": label}
            K = {}
            for levels in (2, 1):
                H = Hierarchy(flowgen.config_paper_cellular(test, scale, n=n_k, levels=levels, divide=5),
                              keep_psi=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                H.run()
                r = H.result()
                rec[f"{'shmm' if levels == 2 else 'direct'}_s"] = round(time.perf_counter() - t0, 3)
                K[levels] = r.K_total[0]
                H.close()
            rec["K_shmm"] = [round(float(v), 6) for v in K[2]]
            rec["K_direct"] = [round(float(v), 6) for v in K[1]]
            rec["rel_gap"] = float(np.max(np.abs(K[2] - K[1])) / K[1][0])
            # direct simulation with the full velocity (face velocities of the one-band filter),
            # recorded at t = 0.02 and t = 0.1 of the paper; the homogenized models alongside
            Hd = Hierarchy(flowgen.config_paper_cellular(test, scale, n=n_dns, levels=1), keep_psi=False)
            Hd.band_filter()
            torch.cuda.synchronize()
            vx, vy = Hd.vx[:n_dns * n_dns].contiguous(), Hd.vy[:n_dns * n_dns].contiguous()
            kap = [1.0, 0.0, 1.0]
            dt, ns = _macro_dt(vx.cpu().numpy(), vy.cpu().numpy(), kap, n_dns, 0.5, T / 5)
            u = torch.tensor(flowgen.paper_step_initial(n_dns), dtype=torch.float32, device="cuda").contiguous()
            Kd = torch.tensor([kap], dtype=torch.float64, device="cuda")
            nm, b = n_dns // 4, 4
            models = {}
            for name, Km in (("shmm", K[2]), ("molecular", np.array(kap))):
                dtm, nsm = _macro_dt(None, None, Km, nm, 0.5, T / 5)
                models[name] = (dtm, nsm, torch.tensor(flowgen.paper_step_initial(nm), dtype=torch.float64,
                                                       device="cuda").contiguous(),
                                torch.tensor([list(Km)], dtype=torch.float64, device="cuda"))
            rec["dns_steps"] = 5 * ns
            rec["dns_s"] = 0.0
            for t_paper, reps in ((0.02, 1), (0.1, 4)):
                t0 = time.perf_counter()
                Hd.ctx.shmm_macro_step(n_dns, abi.BC_DIRICHLET_X, 1.0, 0.0, vx.data_ptr(), vy.data_ptr(),
                                       Kd.data_ptr(), 0, dt, reps * ns, u.data_ptr(), 32, s)
                torch.cuda.synchronize()
                rec["dns_s"] = round(rec["dns_s"] + time.perf_counter() - t0, 3)
                ud = u.cpu().numpy().astype(np.float64).reshape(n_dns, n_dns)
                ubar = ud.mean(axis=0).reshape(nm, b).mean(axis=1)
                at = {"dns_fluctuation_rms": float(np.sqrt(np.mean((ud - ud.mean(axis=0)[None, :]) ** 2)))}
                for name, (dtm, nsm, um, Kt) in models.items():
                    Hd.ctx.shmm_macro_step(nm, abi.BC_DIRICHLET_X, 1.0, 0.0, 0, 0, Kt.data_ptr(), 0, dtm,
                                           reps * nsm, um.data_ptr(), 64, s)
                    torch.cuda.synchronize()
                    prof = um.cpu().numpy().reshape(nm, nm)[nm // 2]
                    at[f"u_rms_vs_dns_{name}"] = float(np.sqrt(np.mean((prof - ubar) ** 2)))
                rec[f"t={t_paper}"] = at
            Hd.close()
            log(f"paper test {test} ({label}): K gap {rec['rel_gap']:.2e}; u rms vs DNS at t = 0.02 / 0.1: "
                f"SHMM {rec['t=0.02']['u_rms_vs_dns_shmm']:.2e} / {rec['t=0.1']['u_rms_vs_dns_shmm']:.2e}, "
                f"kappa alone {rec['t=0.02']['u_rms_vs_dns_molecular']:.2e} / "
                f"{rec['t=0.1']['u_rms_vs_dns_molecular']:.2e}")
            out.append(rec)
    return {"workload": f"Section 4 Tests 2-3: K on wavenumbers / 5 at {n_k}^2; u at t = 0.02 and 0.1 (paper units), "
                        f"DNS {n_dns}^2 FP32, homogenized models {n_dns // 4}^2 FP64",
            "cases": out}


SOLVE_KERNELS_256 = {0: "k_solve_band<256,32,8,16,0>", 1: "k_solve_band<256,32,8,12,0>", 2: "k_solve_stage",
                     3: "k_solve_band<256,24,12,16,0>", 4: "k_solve_band<256,16,8,32,8>",
                     5: "k_solve_tiled<64,8,10>", 6: "k_solve_ring<256,32,8,16>"}


def n256_leg(steps: int = 200):
    """Every kernel variant for 256^2 patches on one phase of 1024 of them (four
    uneven-batch instances at n = 256 with 16 x 16 patches per level), each
    run for `steps` RK4 steps and timed with HIP events on the launch stream
    (best of two)."""
    import torch
    import flowgen
    from paper_1510_00451_amd.hierarchy import Hierarchy
    H = Hierarchy([flowgen.config_batched_instance(100 + i, n=256, lattice=16) for i in range(4)], keep_psi=False)
    H.band_filter()
    H.top_down()
    H.phase_solve(0, steps=1)
    torch.cuda.synchronize()
    first, count = int(H.phase[0]), int(H.phase[1] - H.phase[0])
    table = H.ctx.shmm_ctx_table()[0]
    ns = np.minimum(table["nsteps"][first:first + count].astype(np.int64), steps)
    pts = int(np.sum(table["n"][first:first + count].astype(np.int64) ** 2 * ns))
    a, b = H.cell_range(first, count)
    s = H.stream()
    out = {}
    for v in range(H.ctx.solve_variants(256)):
        H.ctx.shmm_ctx_tune(256, v)
        best = float("inf")
        for rep in range(2):
            H.w.view(2, H.cells)[:, a:b].zero_()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            H.ctx.shmm_local_solve_batch(first, count, H.vx.data_ptr(), H.vy.data_ptr(), H.f1.data_ptr(),
                                         H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(), 0, steps, 0, s)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[SOLVE_KERNELS_256[v]] = round(pts / (best * 1e-3) / 1e9, 1)
        log(f"n = 256 variant {v}: {out[SOLVE_KERNELS_256[v]]} Gpoint-steps/s")
    H.close()
    return {"workload": f"{count} patches of 256^2 (uneven-batch generator, seeds 100-103, n = 256, "
                        f"16 x 16 patches per level), {steps} steps",
            "shortest_plan": int(table["nsteps"][first:first + count].min()),
            "gpoint_steps_per_s": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-flows", type=int, default=64)
    ap.add_argument("--surrogate-eval-flows", type=int, default=32)
    ap.add_argument("--surrogate-steps", type=int, default=1500)
    ap.add_argument("--surrogate-lattice", type=int, default=16)
    ap.add_argument("--no-continuous", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--uneven-instances", type=int, default=256)
    ap.add_argument("--uneven-window", type=int, default=2000)
    ap.add_argument("--no-n256", action="store_true", help="skip the 256^2 kernel-variant leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the Section 4 examples")
    ap.add_argument("--no-oversampling", action="store_true", help="skip the oversampled-patch comparison")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the quasi-stationary-stop passes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy this many MiB once before the passes (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU only: the hot path runs on a single MI355X; patches are "
            "independent, so more GPUs would each take a share of the centres. Use --gpus 1.")
        sys.exit(2)

    import torch
    from paper_1510_00451_amd.hierarchy import Hierarchy
    if not torch.cuda.is_available():
        log("no HIP device: the benchmark needs an MI355X")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        src = torch.full((args.copy_probe_mib << 20,), 1, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    probs = workload()
    H = Hierarchy(probs, keep_psi=False)
    log(f"domains {H.nd}, cells {H.cells}, phases {len(H.phase) - 1}")

    events = []

    def timed_solve(first, count, fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        events.append((first, count, a, b))

    for i in range(max(1, args.warmup)):
        H.run()
        torch.cuda.synchronize()
        log(f"warmup pass {i} done")
        if i == 0:
            from paper_1510_00451_amd import autotune
            tuned = autotune.tune_solve(H, phase=0, steps=300)
            log(f"autotune: {tuned}")
    H.solve_hook = timed_solve
    events.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        H.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    res = H.result()
    log(f"timed {args.steps} passes in {el:.3f} s")

    # per-launch kernel time of the local solves (HIP events on the launch stream)
    table = H.ctx.shmm_ctx_table()[0]
    pts_launch, ms_launch = [], []
    for first, count, a, b in events:
        ms_launch.append(a.elapsed_time(b))
        pts_launch.append(int(np.sum(table["n"][first:first + count].astype(np.int64) ** 2
                                     * table["nsteps"][first:first + count].astype(np.int64))))
    avg_ms = float(np.mean(ms_launch))
    avg_flop = FLOP_PER_POINT_STEP * float(np.mean(pts_launch))
    achieved_tflops = avg_flop / (avg_ms * 1e-3) / 1e12

    pass_pts = res.point_steps
    gpts = pass_pts * args.steps / el / 1e9
    est = H.nd * args.steps / el
    shear_idx = [i for i, d in enumerate(table) if d["instance"] == 1 and d["level"] == 0][0]
    out = {
        "metric": METRIC,
        "value": round(gpts, 3),
        "unit": "Gpoint-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 stencils, f64 reductions",
        "data": "synthetic",
        "config": {"workload": "cellular-4level-64x128 + shear-k16",
                   "levels": 4, "patches_per_level": 64, "n": 128, "kappa": 1e-2,
                   "band_edges": [2, 8, 32], "delta": 1e-6, "dt_frac": 0.5,
                   "point_steps_per_pass": pass_pts, "estimates_per_pass": int(H.nd)},
        "kappa_eff_estimates_per_s": round(est, 2),
        "autotune": {str(k): v for k, v in tuned.items()},
        "K_total_mean": np.mean(res.K_total[:64], axis=0).round(10).tolist(),
        "shear_Kyy": float(res.R[shear_idx][2]),
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": solve_traffic() if tuned.get(128, {"variant": 5})["variant"] == SOLVE_TRAFFIC["variant"]
                     else None,
                     "kernel": SOLVE_KERNELS_128[tuned.get(128, {"variant": 0})["variant"]],
                     "launches": len(ms_launch), "avg_launch_ms": round(avg_ms, 3)},
    }
    if not args.no_adaptive:
        # the same passes with the quasi-stationary stop of HMM step 2
        H.solve_hook = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            H.run(adaptive=True)
        torch.cuda.synchronize()
        el_a = time.perf_counter() - t0
        ra = H.result()
        rel = np.max(np.abs(ra.K_total - res.K_total), axis=1) / np.max(np.abs(res.K_total), axis=1)
        out["adaptive"] = {
            "kappa_eff_estimates_per_s": round(len(ra.R) * args.steps / el_a, 2),
            "ms_per_pass": round(el_a * 1e3 / args.steps, 3),
            "steps_taken_fraction": round(ra.point_steps / res.point_steps, 4),
            "speedup_vs_planned": round(el / el_a, 2),
            "max_rel_K_vs_planned": float(rel.max()),
            "rule": "stop when rms(f) rms(dw) rho/(1-rho) <= delta max|K|, chunks of plan/32"}
        log(f"adaptive: {out['adaptive']}")
    H.close()
    if not args.no_continuous:
        log("continuous-spectrum pass ...")
        out["continuous_5level"] = continuous_leg()
    if not args.no_uneven:
        log("uneven batch ...")
        out["uneven_batch"] = uneven_leg(args.uneven_instances, args.uneven_window)
    if not args.no_n256:
        log("256^2 kernel variants ...")
        out["n256_variants"] = n256_leg()
    if not args.no_paper:
        log("Section 4 examples ...")
        out["paper_tests"] = paper_tests_leg()
    if not args.no_oversampling:
        log("oversampled patches ...")
        out["oversampling"] = oversampling_leg()
    if not args.no_surrogate:
        log("surrogate ...")
        out["surrogate"] = surrogate_leg(args.surrogate_flows, args.surrogate_eval_flows,
                                         steps=args.surrogate_steps, lattice=args.surrogate_lattice)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the TTCF daughter path on one MI355X.

Workload (the batched bulk configuration): WCA fluid, N = 2048 (8^3 fcc cells), rho = 0.8442,
T = 0.722, dt = 0.0025. One Nose-Hoover mother (melted at T = 2 for 1000 steps, equilibrated
2000 steps) is sampled every 100 steps into 1024 start states that stay resident in HBM. A
benchmark step is one pass of the daughter path over one batch: spawn the 4 mapped daughters
of every start state (4096 daughters), run 500 isokinetic SLLOD steps each in one persistent
launch (FP32 pair forces, FP64 integration), accumulate, and form the TTCF response. The
shear rate cycles through {1e-6, 1e-4, 1e-2, 1} from step to step.

Prints one JSON line; ``value`` is daughter atom-steps per second over the timed steps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "daughter atom-steps/s; TTCF σ(P_xy) per GPU-s, learned CV vs plain"
HBM_PEAK_GBS = 8000.0
BYTES_PER_ATOM_STEP = 96  # read and write of r and p in FP64 (6 x 8 B each way)
GAMMAS = (1e-6, 1e-4, 1e-2, 1.0)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_daughters_config2_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "k_daughters_config2_valu.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2312_02990_amd", "csrc", "ttcf_pairs.hip")
PEF_SRC = os.path.join(ROOT, "paper_2312_02990_amd", "csrc", "ttcf_elongation.hip")
PEF_VALU_FILE = os.path.join(ROOT, "profiles", "k_daughters_pef_n2048_valu.json")
MIX_VALU_FILE = os.path.join(ROOT, "profiles", "k_daughters_mix_n2048_valu.json")
CH_SRC = os.path.join(ROOT, "paper_2312_02990_amd", "csrc", "ttcf_channel.hip")
CH_VALU_FILE = os.path.join(ROOT, "profiles", "k_channel_config4_valu.json")
LANE_SLOT_PEAK = 256 * 4 * 16 * 2.4e9  # VALU lane-instruction slots per second


_T0 = time.perf_counter()


def progress(what: str):
    """One line on stderr per finished part (the JSON line alone goes to stdout)."""
    print(f"bench: {what} done at {time.perf_counter() - _T0:.0f} s", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were taken on
    the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def measured_valu():
    """VALU figures of the step kernel from the committed SQ counter runs, if they were taken
    on the current kernel source; otherwise None. The kernel keeps its state on chip, so its
    bound is VALU issue rather than HBM."""
    try:
        with open(VALU_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return {k: rec[k] for k in ("valu_busy", "lane_slots_issued_frac", "active_lanes",
                                "lane_slots_per_atom_step") if k in rec}


def host_threads() -> int:
    """Threads of the CPU baseline: the cores this process may run on, at most 16 (a one-GPU
    box's share of the host; nproc may show more)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_description() -> dict:
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"nproc": os.cpu_count(), "affinity": affinity, "threads_used_max": host_threads(),
            "model": cpu_model()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_cells: int, nsteps: int, budget_s: float, states=None):
    """The FP64 oracle, unchanged, on a bounded sample of the same workload: the first start
    states of the GPU batch (`states` = (r, p), as exported from the mother), their four
    mapped daughters each, at one shear rate, one daughter per thread at a time on the host's
    cores. Without `states`, seeded perturbed-lattice start states."""
    import oracle as orc
    import ttcf_inputs as I
    s = I.System(n_cells)
    box = orc.make_box(s.n, s.box)
    threads = host_threads()
    # calibrate: one daughter, a few steps, one thread
    r = I.perturbed_positions(s, 5, 0.1).reshape(1, -1)
    p = I.maxwell_boltzmann(s.n, s.temperature, 5).reshape(1, -1)
    t0 = time.perf_counter()
    orc.run_daughters(box, r, p, [0], [0], [1e-2], s.dt, 20, nthreads=1)
    per_step = (time.perf_counter() - t0) / 20
    per_daughter = per_step * nsteps
    n_d = max(threads, int(budget_s * threads / per_daughter) // threads * threads)
    n_states = (n_d + 3) // 4
    if states is not None and len(states[0]) >= n_states:
        sr, sp = states[0][:n_states], states[1][:n_states]
        origin = "the GPU batch's first start states"
    else:
        sr = np.stack([I.perturbed_positions(s, 100 + k, 0.1).ravel() for k in range(n_states)])
        sp = np.stack([I.maxwell_boltzmann(s.n, s.temperature, 100 + k).ravel()
                       for k in range(n_states)])
        origin = "seeded perturbed-lattice start states"
    state_of = np.arange(n_d) // 4
    map_of = np.arange(n_d) % 4
    t0 = time.perf_counter()
    _, used = orc.run_daughters(box, sr, sp, state_of, map_of, np.full(n_d, 1e-2), s.dt, nsteps,
                                nthreads=threads)
    dt = time.perf_counter() - t0
    return {
        "value": n_d * s.n * nsteps / dt, "unit": "daughter atom-steps/s", "cores": int(used),
        "kind": "oracle",
        "sample": f"{n_d} daughters x {nsteps} steps of the N={s.n} system from {origin} "
                  f"(FP64 oracle, {used} threads on {cpu_model()}), {dt:.1f} s",
        "host": host_description(),
    }


def cpu_baseline_configs(seed=41):
    """The oracle on bounded samples of the other workloads, same threads: the plain FP64
    workload (N = 256, 32 daughters x 100 steps, all of it), the uneven batch (8 daughters of
    each size x 100 of its 400 steps), the channel (64 daughters x 2 of its 1000 steps, all
    from one lattice start state) and the control-variate workload (N = 256, 64 daughters x 200
    steps, and the network's forward and backward pass over 1024 rows in FP64 numpy). Rates in
    atom-steps per second (rows per second for the network)."""
    import oracle as orc
    import oracle.channel as och
    import oracle.mlp as omlp
    import ttcf_inputs as I
    threads = host_threads()
    out = {"threads": threads}

    def daughters(s, n_d, nsteps, gammas, sd):
        box = orc.make_box(s.n, s.box)
        n_states = (n_d + 3) // 4
        sr = np.stack([I.perturbed_positions(s, sd + k, 0.1).ravel() for k in range(n_states)])
        sp = np.stack([I.maxwell_boltzmann(s.n, s.temperature, sd + k).ravel()
                       for k in range(n_states)])
        t0 = time.perf_counter()
        orc.run_daughters(box, sr, sp, np.arange(n_d) // 4, np.arange(n_d) % 4, gammas, s.dt,
                          nsteps, nthreads=threads)
        return n_d * s.n * nsteps / (time.perf_counter() - t0)

    s1 = I.System(4)
    out["config1_plain_fp64"] = {"value": daughters(s1, 32, 100, np.full(32, 1e-3), seed),
                                 "sample": "32 daughters x 100 steps, N=256 (the whole workload)"}
    rng = np.random.Generator(np.random.PCG64(seed))
    per_size = {}
    for n_cells, rho in ((5, 0.7), (6, 0.8442), (8, 0.9), (10, 0.7)):
        s = I.System(n_cells, density=rho)
        g = np.exp(rng.uniform(np.log(1e-5), np.log(1e-1), 8))
        per_size[str(s.n)] = daughters(s, 8, 100, g, seed + n_cells)
    out["config3_uneven"] = {"per_size": per_size,
                             "sample": "8 daughters x 100 steps per size, rates log-uniform in "
                                       "[1e-5, 1e-1]"}
    g = I.ChannelSystem()
    ch = och.make_channel(g)
    r, p, lat = I.channel_initial_state(g, seed)
    n_d, nsteps = 64, 2
    q = och.nh_q(g.n_wall, g.temperature, g.nh_tau)
    t0 = time.perf_counter()
    och.run_daughters(ch, r.reshape(1, -1), p.reshape(1, -1), np.zeros(1), lat,
                      np.zeros(n_d, np.int32), np.arange(n_d) % 4, np.full(n_d, 1e-2),
                      g.temperature, q, g.dt, nsteps, nthreads=threads)
    out["config4_channel"] = {"value": n_d * g.n * nsteps / (time.perf_counter() - t0),
                              "sample": f"{n_d} daughters x {nsteps} steps of the {g.n}-atom "
                                        "channel from one lattice start state"}
    out["config5_cv_daughters"] = {"value": daughters(s1, 64, 200, np.full(64, 1e-4), seed + 99),
                                   "sample": "64 daughters x 200 steps, N=256, rate 1e-4"}
    net = omlp.init_weights(64, 256, 200, seed)
    x = np.random.Generator(np.random.PCG64(seed)).standard_normal((1024, 64))
    t = np.zeros((1024, 200))
    t0 = time.perf_counter()
    for _ in range(5):
        y, cache = omlp.forward(net, x)
        omlp.backward(net, cache, y, t)
    out["config5_mlp_rows_per_s"] = {"value": 5 * 1024 / (time.perf_counter() - t0),
                                     "sample": "forward and backward of 64-256-256-200 over "
                                               "1024 rows, 5 times, FP64 numpy"}
    return out


def per_rate_statement(responses, expected, nst, dt):
    """Per shear rate of the sweep: the TTCF and direct-average (DAV) responses of P_xy at the
    last time point with their block standard errors, the healthy groups against the groups
    run (a rate's response covers every batch run at it), the standard errors per start state
    over the rate, SE sqrt(groups) / gamma_dot (Eq. variance: for TTCF it is the same at every
    rate of the linear regime; the mapped direct average cancels its equilibrium part too, so
    its error also falls with the rate until the mapped trajectories stop mirroring each
    other), and the largest |TTCF - DAV| over time in combined standard errors."""
    out = {}
    for gd in sorted(responses):
        tm, tse, dm, dse, used = responses[gd]
        comb = np.hypot(tse, dse)[1:]
        root = np.sqrt(max(int(used), 1))
        out[str(gd)] = {
            "groups": int(used), "groups_expected": int(expected[gd]),
            "ttcf_end": float(tm[-1]), "ttcf_se_end": float(tse[-1]),
            "dav_end": float(dm[-1]), "dav_se_end": float(dse[-1]),
            "ttcf_se_per_state_over_rate_end": float(tse[-1] * root / gd),
            "dav_se_per_state_over_rate_end": float(dse[-1] * root / gd),
            "max_abs_ttcf_minus_dav_over_se": float(np.max(np.abs(tm[1:] - dm[1:]) / comb)),
            "t_end": nst * dt,
        }
    small = [g for g in responses if g < 1.0]  # the linear-response part of the sweep
    ratio = lambda v: float(max(v) / min(v)) if v and min(v) > 0 else None
    summary = {
        "ttcf_se_per_state_over_rate_max_over_min_linear":
            ratio([out[str(g)]["ttcf_se_per_state_over_rate_end"] for g in small]),
        "all_groups_healthy": all(int(responses[g][4]) == expected[g] for g in responses),
    }
    return {"rates": out, "summary": summary}


def precision_statement(T, ctx, mid, sysd, s, n_states, nst, stream):
    """FP32-force responses against FP64-force responses (the paper's arithmetic) from the
    same start states, at each shear rate: max over t of |difference| in units of the FP64
    response's standard error, and relative to the largest |TTCF|. Both reruns step all four
    rates' daughters in one call, timed: the throughput of each arithmetic on the same
    workload, with the roofline fraction of the headline (96 B per atom-step)."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    sys64 = T.make_system(s.n, s.box, s.temperature, s.dt, precision=0)
    out, rates = {}, {}
    atom_steps = 4 * n_states * len(GAMMAS) * s.n * nst
    for prec, tag in ((1, "fp32"), (0, "fp64")):
        res = {}
        with T.Context(stream) as c2:
            sysp = sysd if prec == 1 else sys64
            m2 = c2.ttcf_init_mother(sysp, r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            for gd in GAMMAS:
                c2.ttcf_spawn_daughters(m2, n_states, 0, gd, nst)
            torch.cuda.synchronize()
            c2.ttcf_step_timing(reset=True)
            t0 = time.perf_counter()
            c2.ttcf_step(nst)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms, launches = c2.ttcf_step_timing(reset=True)
            c2.ttcf_accumulate()
            for gd in GAMMAS:
                res[gd] = c2.ttcf_response(nst + 1, gd)
        out[tag] = res
        achieved = BYTES_PER_ATOM_STEP * atom_steps / (ms / 1e3) / 1e9
        rates[tag] = {
            "atom_steps_per_s": atom_steps / wall,
            "kernel_atom_steps_per_s": atom_steps / (ms / 1e3),
            "kernel_ms": ms, "launches": int(launches),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
            "workload": f"{4 * n_states * len(GAMMAS)} daughters (all four rates) x {nst} "
                        f"steps of N={s.n} in one step call",
        }
    stmt = {}
    for gd in GAMMAS:
        a, b = out["fp32"][gd], out["fp64"][gd]
        k = slice(1, None)
        stmt[str(gd)] = {
            "ttcf_max_err_over_se": float(np.max(np.abs(a[0][k] - b[0][k]) / b[1][k])),
            "ttcf_max_rel_err": float(np.max(np.abs(a[0] - b[0])) / np.max(np.abs(b[0]))),
            "dav_max_err_over_se": float(np.max(np.abs(a[2][k] - b[2][k]) / b[3][k])),
        }
    return {"reference": "same start states, FP64 pair forces (the FP64 form matches the "
                         "oracle to 1e-9 over 50 steps)", "per_shear_rate": stmt,
            "throughput": rates}


def uneven_leg(T, stream, sizes=(5, 6, 8, 10), densities=(0.7, 0.8442, 0.9), per_size=128,
               nst=400, seed=31, tune=True):
    """Mixed system sizes in one step call: N in {500, 864, 2048, 4000} x rho in {0.7, 0.8442,
    0.9}, one mother per (N, rho), 128 start states per N (state n at density index n mod 3),
    a shear rate per state drawn log-uniformly in [1e-5, 1e-1] (shared by its four mapped
    daughters), 400 steps, FP32 forces. Start states come from replicas of each mother
    (kicked, decorrelated). The response is the per-unit-rate TTCF over all groups."""
    import torch
    import ttcf_inputs as I
    ctx = T.Context(stream)
    t0 = time.perf_counter()
    total_atoms = 0
    spawned = []
    shapes = {}
    tune_s = 0.0
    rates = I.log_uniform_rates(len(sizes) * per_size, 1e-5, 1e-1, seed)
    ri = 0
    for nc in sizes:
        for di, rho in enumerate(densities):
            count = len([k for k in range(per_size) if k % len(densities) == di])
            s = I.System(nc, density=rho)
            r0, p0 = I.initial_state(s, 3000 + 10 * nc + di)
            mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                       r0, p0, n_equil=1000, n_melt=1000, t_melt=2.0)
            n_rep = count
            ctx.ttcf_sample_states_replicated(mid, n_rep, seeded_kicks(n_rep, s.n, 0.05, seed + mid),
                                              200, 1, 50)
            if tune:
                t1 = time.perf_counter()
                sh = ctx.ttcf_autotune(mid, 0, 1e-3, 200)
                tune_s += time.perf_counter() - t1
                shapes[f"N={s.n} rho={rho}"] = (
                    f"{'lists' if sh['variant'] == 2 else 'cells'}/{sh['threads']}"
                    + (f" skin {sh['skin']:.3f} kmax {sh['kmax']}" if sh["variant"] == 2 else ""))
            spawned.append((mid, count, s.n, rates[ri:ri + count]))
            ri += count
    torch.cuda.synchronize()
    mother_s = time.perf_counter() - t0 - tune_s
    for mid, count, n, g in spawned:
        ctx.ttcf_spawn_daughters(mid, count, 0, g, nst)
        total_atoms += 4 * count * n
    ctx.ttcf_step_timing(reset=True)
    t0 = time.perf_counter()
    ctx.ttcf_step(nst)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, launches = ctx.ttcf_step_timing(reset=True)
    groups = ctx.ttcf_accumulate()
    tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, 0.0)
    atom_steps = total_atoms * nst
    # each size alone (the same states and rates, one step call per size)
    per_size_rate = {}
    for nc in sizes:
        n = 4 * nc ** 3
        mine = [(mid, count, g) for mid, count, nn, g in spawned if nn == n]
        for mid, count, g in mine:
            ctx.ttcf_spawn_daughters(mid, count, 0, g, nst)
        ctx.ttcf_step_timing(reset=True)
        ctx.ttcf_step(nst)
        ms1, _ = ctx.ttcf_step_timing(reset=True)
        ctx.ttcf_accumulate()
        per_size_rate[str(n)] = 4 * sum(c for _, c, _ in mine) * n * nst / (ms1 / 1e3)
    # the same batch as one captured cycle over all twelve mothers: each replay runs the
    # mothers' kicked copies (one state each, 50 steps), spawns, steps and accumulates
    parts = [{"mother": mid, "n_replicas": count, "states_per_replica": 1, "steps_between": 50,
              "gamma_dot": g, "kicks": seeded_kicks(count, n, 0.05, seed + 100 + mid),
              "decorrelate_steps": 200} for mid, count, n, g in spawned]
    replays = 2
    gr = ctx.ttcf_graph_create_multi(parts, nst, replays + 1)
    gr.launch(1)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr.launch(replays)
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / replays
    g_resp = ctx.ttcf_response(nst + 1, 0.0)
    ctx.close()
    return {"workload": f"sizes {[4 * n ** 3 for n in sizes]} x densities {list(densities)}, "
                        f"{per_size} states per size x 4 mappings, {nst} steps, per-state shear "
                        f"rates log-uniform in [1e-5, 1e-1]",
            "daughters": 4 * len(sizes) * per_size, "kernel_launches": launches,
            "kernel_atom_steps_per_s": atom_steps / (ms / 1e3),
            "end_to_end_atom_steps_per_s": atom_steps / wall, "mothers_s": mother_s,
            "autotune_s": tune_s, "tuned_shapes": shapes,
            "healthy_groups": int(groups),
            "per_unit_rate_ttcf_end": float(tm[-1]), "per_unit_rate_ttcf_se_end": float(tse[-1]),
            "per_size_kernel_atom_steps_per_s": per_size_rate,
            "captured": {"ms_per_cycle": 1e3 * graph_s,
                         "daughter_atom_steps_per_s": atom_steps / graph_s,
                         "mother_atom_steps_per_cycle": sum(c * n * 50 for _, c, n, _ in spawned),
                         "groups_after_replays": int(g_resp[4]),
                         "cycle": "12 mothers' kicked copies (one state each, 50 steps) -> spawn "
                                  "-> one step per kernel form -> accumulate, one HIP graph"}}


def thermostat_leg(T, stream, ctx, mid, s, n_states, nst, gd=1e-2):
    """Gaussian isokinetic against Nose-Hoover daughters (the paper's own dynamics, zeta
    carried from each start state) on the benchmark's 1024 start states at one shear rate:
    TTCF and direct average at the end, and the step kernel's throughput for each."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    z = ctx.ttcf_export_states_zeta(mid, n_states)
    out = {"gamma_dot": gd, "workload": f"N={s.n}, {n_states} states x 4 mappings x {nst} steps"}
    for name, th in (("gik", 0), ("nose_hoover", 1)):
        with T.Context(stream) as c2:
            m2 = c2.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1,
                                                   thermostat=th), r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            c2.ttcf_import_states_zeta(m2, z)
            c2.ttcf_spawn_daughters(m2, n_states, 0, gd, nst)
            c2.ttcf_step_timing(reset=True)
            c2.ttcf_step(nst)
            ms, _ = c2.ttcf_step_timing(reset=True)
            c2.ttcf_accumulate()
            tm, tse, dm, dse, used = c2.ttcf_response(nst + 1, gd)
            torch.cuda.synchronize()
        out[name] = {"ttcf_end": float(tm[-1]), "ttcf_se_end": float(tse[-1]),
                     "dav_end": float(dm[-1]), "dav_se_end": float(dse[-1]),
                     "kernel_atom_steps_per_s": 4 * n_states * s.n * nst / (ms / 1e3)}
    a, b = out["gik"], out["nose_hoover"]
    out["ttcf_difference_over_se"] = (a["ttcf_end"] - b["ttcf_end"]) / float(
        np.hypot(a["ttcf_se_end"], b["ttcf_se_end"]))
    return out


def green_kubo_leg(T, ctx, mid, s, n_samples, nst, gd=1e-4, resp_ctx=None):
    """Weak-field check at full size: the TTCF viscosity eta(t) = -TTCF(t)/gamma_dot of the
    benchmark's groups at gamma_dot = 1e-4 against the Green-Kubo integral
    (V/T) int_0^t <P_xy(0) P_xy(s)> ds of the mother's recorded V P_xy (the series the start
    states were sampled from), both at t = 0.25, 0.5 and the daughters' end. resp_ctx: the
    context that holds the benchmark's groups at gamma_dot (ctx when None)."""
    vp = ctx.ttcf_export_mother_series(mid, n_samples)
    acf, _, _ = ctx.ttcf_mother_acf(mid, nst + 1, 0.05)
    cov = acf * float(np.var(vp))                       # <VP(0) VP(t)>, mean removed
    gk = np.concatenate([[0.0], np.cumsum(0.5 * s.dt * (cov[1:] + cov[:-1]))])
    gk /= s.volume * s.temperature
    tm, tse, dm, dse, used = (ctx if resp_ctx is None else resp_ctx).ttcf_response(nst + 1, gd)
    out = {"gamma_dot": gd, "n_states": used, "mother_samples": n_samples}
    for k in (100, 200, nst):
        out[f"t={k * s.dt:g}"] = {"eta_ttcf": float(-tm[k] / gd), "eta_ttcf_se": float(tse[k] / gd),
                                  "eta_green_kubo": float(gk[k])}
    return out


def observables_leg(T, stream, ctx, mid, s, n_states, nst, gd=1e-2):
    """The benchmark's start states run once more with the extra bulk observables recorded
    (P_xx - P_yy, P_yy - P_zz, energy per atom, y-slab momentum profile): the step kernel's
    throughput with and without them, and each observable's TTCF and direct average at the
    end (the slab profile as its largest magnitude over the slabs)."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    out = {"gamma_dot": gd, "workload": f"N={s.n}, {n_states} states x 4 mappings x {nst} steps"}
    rates = {}
    for rec in (False, True):
        with T.Context(stream) as c2:
            m2 = c2.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                     r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            c2.ttcf_record_observables(rec)
            c2.ttcf_spawn_daughters(m2, n_states, 0, gd, nst)
            c2.ttcf_step_timing(reset=True)
            c2.ttcf_step(nst)
            ms, _ = c2.ttcf_step_timing(reset=True)
            rates[rec] = 4 * n_states * s.n * nst / (ms / 1e3)
            if rec:
                c2.ttcf_accumulate()
                for name, o in (("n1", T.TTCF_OBS_N1), ("n2", T.TTCF_OBS_N2),
                                ("energy_per_atom", T.TTCF_OBS_ENERGY),
                                ("slab_px", T.TTCF_OBS_SLAB_PX)):
                    tm, tse, dm, dse, _ = c2.ttcf_response(nst + 1, gd, observable=o)
                    tm, tse, dm, dse = [np.atleast_2d(np.asarray(x).T).T for x in (tm, tse, dm, dse)]
                    q = int(np.argmax(np.abs(tm[-1])))
                    out[name] = {"ttcf_end": float(tm[-1, q]), "ttcf_se_end": float(tse[-1, q]),
                                 "dav_end": float(dm[-1, q]), "dav_se_end": float(dse[-1, q])}
            torch.cuda.synchronize()
    out["kernel_atom_steps_per_s"] = rates[True]
    out["kernel_atom_steps_per_s_without"] = rates[False]
    out["cost_ratio"] = rates[False] / rates[True]
    return out


def colour_leg(T, stream, ctx, mid, s, n_states, nst, fields=(1e-2, 1e-4)):
    """The benchmark's start states under the colour field instead of shear (charge +1 on
    even atoms, -1 on odd ones): colour conductivity sigma(t) = <J_x(t)>/F_e by TTCF and by
    the direct average at the end, with standard errors, and the kernel's throughput."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    out = {"workload": f"N={s.n}, {n_states} states x 4 mappings x {nst} steps per field"}
    for fe in fields:
        with T.Context(stream) as c2:
            m2 = c2.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                     r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            c2.ttcf_spawn_colour(m2, n_states, 0, fe, nst)
            c2.ttcf_step_timing(reset=True)
            c2.ttcf_step(nst)
            ms, _ = c2.ttcf_step_timing(reset=True)
            c2.ttcf_accumulate()
            tm, tse, dm, dse, used = c2.ttcf_response(nst + 1, 0.0, observable=T.TTCF_OBS_JX)
            torch.cuda.synchronize()
        out[f"F_e={fe:g}"] = {"sigma_ttcf_end": float(tm[-1]), "sigma_ttcf_se_end": float(tse[-1]),
                              "sigma_dav_end": float(dm[-1]), "sigma_dav_se_end": float(dse[-1]),
                              "n_states": used,
                              "kernel_atom_steps_per_s": 4 * n_states * s.n * nst / (ms / 1e3)}
    return out


def pef_roofline(kernel_ms, atom_steps, valu_file=PEF_VALU_FILE):
    """FP64 roofline of the planar-elongation (or mixed-flow) kernel: the FP64 lane
    operations per atom-step from the committed SQ counter run (while the kernel source
    matches it) over the live kernel time, against the FP64 vector peak."""
    try:
        with open(valu_file) as f:
            rec = json.load(f)
        with open(PEF_SRC, "rb") as f:
            if rec.get("kernel_sha256_16") != hashlib.sha256(f.read()).hexdigest()[:16]:
                return None
    except (OSError, ValueError):
        return None
    flops = rec["fp64_flops_per_launch"] / rec["atom_steps_per_launch"] * atom_steps
    achieved = flops / (kernel_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
            "frac": achieved / 78.6, "traffic": None, "valu_busy": rec["valu_busy"],
            "counts": "FP64 lane operations issued (FMA = 2, masked lanes included), from "
                      + rec["source"]}


def elongation_leg(T, stream, ctx, mid, s, n_states, nst, rates=(1.0, 1e-2, 1e-4)):
    """The benchmark's start states under planar elongational flow instead of shear
    (grad u = diag(rate, -rate, 0), mappings: identity, reversed momenta, x and y exchanged,
    both): -<P_xx - P_yy>(t) / (4 rate), the elongational viscosity over 4 (the shear
    viscosity in the linear regime), by TTCF and by the direct average at t = 0.25 and at
    the end, with standard errors, and the FP64 kernel's throughput."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    out = {"workload": f"N={s.n}, {n_states} states x 4 mappings x {nst} steps per rate"}
    for rate in rates:
        with T.Context(stream) as c2:
            m2 = c2.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                     r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            c2.ttcf_spawn_elongational(m2, n_states, 0, rate, nst)
            c2.ttcf_step_timing(reset=True)
            c2.ttcf_step(nst)
            ms, _ = c2.ttcf_step_timing(reset=True)
            c2.ttcf_accumulate()
            tm, tse, dm, dse, used = c2.ttcf_response(nst + 1, rate,
                                                      observable=T.TTCF_OBS_PEF_N1)
            torch.cuda.synchronize()
        f = -1.0 / (4.0 * rate)
        row = {"n_states": used, "kernel_ms": ms,
               "kernel_atom_steps_per_s": 4 * n_states * s.n * nst / (ms / 1e3)}
        for k in (100, nst):
            row[f"t={k * s.dt:g}"] = {"eta_ttcf": float(f * tm[k]), "eta_ttcf_se": float(-f * tse[k]),
                                      "eta_dav": float(f * dm[k]), "eta_dav_se": float(-f * dse[k])}
        out[f"rate={rate:g}"] = row
    ms = [out[k]["kernel_ms"] for k in out if k.startswith("rate=")]
    out["roofline"] = pef_roofline(sum(ms) / len(ms), 4 * n_states * s.n * nst)
    return out


def mixed_leg(T, stream, ctx, mid, s, n_states, nst, pair=(0.5, 1.0), scales=(1.0, 1e-2, 1e-4)):
    """The benchmark's start states under mixed flow (u_x = erate x + srate y,
    u_y = -erate y, the pair scaled down): the generalised viscosity
    -<J> |rate| / (4 erate^2 + srate^2) (the shear viscosity for a Newtonian fluid) by TTCF
    and by the direct average at t = 0.25 and at the end, and the FP64 kernel's throughput."""
    import torch
    r, p = ctx.ttcf_export_states(mid, n_states)
    out = {"workload": f"N={s.n}, {n_states} states x 4 mappings x {nst} steps per rate pair"}
    for sc in scales:
        er, sr = pair[0] * sc, pair[1] * sc
        rn = float(np.sqrt(er * er + sr * sr))
        with T.Context(stream) as c2:
            m2 = c2.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                     r[0], p[0], n_equil=0)
            c2.ttcf_import_states(m2, r, p)
            c2.ttcf_spawn_mixed(m2, n_states, 0, er, sr, nst)
            c2.ttcf_step_timing(reset=True)
            c2.ttcf_step(nst)
            ms, _ = c2.ttcf_step_timing(reset=True)
            c2.ttcf_accumulate()
            tm, tse, dm, dse, used = c2.ttcf_response(nst + 1, rn, observable=T.TTCF_OBS_MIX_J)
            torch.cuda.synchronize()
        f = -rn / (4.0 * er * er + sr * sr)
        row = {"erate": er, "srate": sr, "n_states": used, "kernel_ms": ms,
               "kernel_atom_steps_per_s": 4 * n_states * s.n * nst / (ms / 1e3)}
        for k in (100, nst):
            row[f"t={k * s.dt:g}"] = {"eta_ttcf": float(f * tm[k]), "eta_ttcf_se": float(-f * tse[k]),
                                      "eta_dav": float(f * dm[k]), "eta_dav_se": float(-f * dse[k])}
        out[f"scale={sc:g}"] = row
    ms = [out[k]["kernel_ms"] for k in out if k.startswith("scale=")]
    out["roofline"] = pef_roofline(sum(ms) / len(ms), 4 * n_states * s.n * nst, MIX_VALU_FILE)
    return out


def graph_leg(T, stream, n_cells=8, copies=1024, between=100, nst=500, gd=1e-2, replays=3,
              decorrelate=400, seed=7):
    """Whole batch cycles replayed from one captured graph: 1024 persistent copies of the
    N = 2048 mother (kicked, decorrelated 400 steps) each advance 100 steps and save one start
    state, whose four mapped daughters run 500 steps at shear rate 1e-2 and are folded into
    the accumulator, with no host work between replays. Throughput counts daughter atom-steps
    only, while the timed cycle also holds the mother steps, spawn and accumulation."""
    import torch
    import ttcf_inputs as I
    s = I.System(n_cells)
    r0, p0 = I.initial_state(s, 2)
    with T.Context(stream) as ctx:
        mid = ctx.ttcf_init_mother(T.make_system(s.n, s.box, s.temperature, s.dt, precision=1),
                                   r0, p0, n_equil=2000, n_melt=1000, t_melt=2.0)
        g = ctx.ttcf_graph_create(mid, 1, between, gd, nst, max_replays=replays + 1,
                                  n_replicas=copies, kicks=seeded_kicks(copies, s.n, 0.05, seed),
                                  decorrelate_steps=decorrelate)
        g.launch(1)  # warm-up replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch(replays)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm, tse, dm, dse, used = ctx.ttcf_response(nst + 1, gd)
    atom_steps = 4 * copies * s.n * nst * replays
    return {"workload": f"N={s.n} WCA, {copies} mother copies x 1 state per replay ({between} "
                        f"steps apart), 4 mappings x {nst} steps at shear rate {gd}; "
                        f"{replays} timed replays",
            "ms_per_cycle": 1e3 * wall / replays,
            "daughter_atom_steps_per_s": atom_steps / wall,
            "mother_atom_step_share": between / (between + 4 * nst),
            "n_states": int(used), "ttcf_end": float(tm[-1]), "ttcf_se_end": float(tse[-1]),
            "dav_end": float(dm[-1]), "dav_se_end": float(dse[-1])}


def channel_leg(T, stream, n_states=256, nst=1000, speeds=(1e-2, 1e-4), n_equil=2000,
                between=20, seed=4, decorrelate=200, kick=0.05):
    """The confined channel at full size: 12000 fluid + 2 x 3000 tethered wall atoms, LJ
    with wetting factors 1.2 / 0.6325, r_c = 2.5, k = 150, wall thermostat at T = 1,
    dt = 0.005. One mother equilibrates n_equil steps; n_states kicked copies of it then run
    `decorrelate` + `between` steps in one launch and each saves one start state (the paper
    samples one mother 5 time units apart); each lattice speed gets n_states x 4 daughters
    of nst steps in one launch."""
    import torch
    import ttcf_inputs as I
    g = I.ChannelSystem()
    r, p, lat = I.channel_initial_state(g, seed)
    out = {"workload": f"channel: {g.n_fluid} fluid + {g.n_wall} wall atoms, lx={g.lx:.2f}, "
                       f"lz={g.lz:.2f}, gap={g.gap:.2f}; {n_states} states x 4 mappings x "
                       f"{nst} steps per lattice speed, speeds {list(speeds)}"}
    with T.ChannelContext(T.make_channel(g), r, p, lat, stream) as ctx:
        t0 = time.perf_counter()
        ctx.run_mother(n_equil)
        torch.cuda.synchronize()
        serial_s = time.perf_counter() - t0
        ctx.sample_states_replicated(n_states, seeded_kicks(n_states, g.n, kick, seed + 1),
                                     decorrelate, 1, between)
        torch.cuda.synchronize()
        out["mother_s"] = time.perf_counter() - t0
        out["mother_serial_s"] = serial_s
        out["mother_replicas"] = {"copies": n_states, "kick": kick, "decorrelate_steps": decorrelate,
                                  "steps_between": between,
                                  "atom_steps_per_s": n_states * (decorrelate + between) * g.n /
                                  (out["mother_s"] - serial_s)}
        out["mother_atom_steps_per_s"] = n_equil * g.n / serial_s
        ctx.step_timing(reset=True)
        t0 = time.perf_counter()
        for v in speeds:
            ctx.spawn(n_states, v, nst)
            ctx.step(nst)
            ctx.accumulate()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, launches = ctx.step_timing(reset=True)
        atom_steps = len(speeds) * 4 * n_states * nst * g.n
        out["kernel_atom_steps_per_s"] = atom_steps / (ms / 1e3)
        out["end_to_end_atom_steps_per_s"] = atom_steps / wall
        out["kernel_ms_per_launch"] = ms / max(launches, 1)
        out["roofline"] = channel_roofline(atom_steps / (ms / 1e3))
        resp = {}
        for v in speeds:
            tm, tse, dm, dse, used = ctx.response(T.TTCF_OBS_WALL_STRESS, v, nst + 1)
            pm, pse, pd, _, _ = ctx.response(T.TTCF_OBS_VPROFILE, v, nst + 1)
            filled = np.nonzero(np.abs(pd).max(axis=0) > 0)[0]  # bins the fluid reaches
            lo, hi = (int(filled[0]), int(filled[-1])) if filled.size else (0, 0)
            resp[str(v)] = {"wall_stress_ttcf_end": float(tm[-1]), "se": float(tse[-1]),
                            "wall_stress_dav_end": float(dm[-1]), "dav_se": float(dse[-1]),
                            "profile_bins_filled": [lo, hi],
                            "profile_ttcf_end_edge_bins": [float(pm[-1, lo]), float(pm[-1, hi])],
                            "profile_se_end_edge_bins": [float(pse[-1, lo]), float(pse[-1, hi])],
                            "n_states": int(used)}
        out["responses"] = resp
    return out


def channel_roofline(atom_steps_per_s: float):
    """The channel kernel is bound by VALU issue (FP32 LJ pair forces at r_c = 2.5): the lane
    slots it issues per second (its measured slots per atom-step, from the committed SQ counter
    runs on the current source, times the live rate) against the chip's 3.93e13 (256 CUs x 4
    SIMDs x 16 lanes x 2.4 GHz). None without a matching counter run."""
    try:
        with open(CH_VALU_FILE) as f:
            rec = json.load(f)
        with open(CH_SRC, "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != cur:
        return None
    achieved = rec["lane_slots_per_atom_step"] * atom_steps_per_s
    return {"bound": "alu", "achieved": achieved, "peak": LANE_SLOT_PEAK, "unit": "lane-slots/s",
            "frac": achieved / LANE_SLOT_PEAK, "valu_busy": rec.get("valu_busy"),
            "active_lanes": rec.get("active_lanes"),
            "lane_slots_per_atom_step": rec["lane_slots_per_atom_step"], "traffic": None}


def seeded_kicks(n_rep: int, n: int, scale: float, seed: int):
    """Zero-sum momentum kicks, one set per mother copy (numpy PCG64, seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = scale * rng.standard_normal((n_rep, 3, n))
    k -= k.mean(axis=2, keepdims=True)
    return k.reshape(n_rep, 3 * n)


def cv_leg(T, stream, gd=1e-4, nst=200, train_states=4096, eval_states=4096, epochs=30,
           batch=256, lr=1e-3, mean_replicas=1024, mean_rounds=20, mean_per_round=49,
           mean_between=50, decorrelate=400, kick=0.05, seed=5, verbose=False):
    """Learned control variate on the config-5 workload: WCA N=256 at the paper's state
    point, shear rate 1e-4, daughters of 200 steps. Training daughters, evaluation daughters
    and the mean-term samples come from separate branches of one mother (copies kicked by
    seeded zero-sum momentum changes, then decorrelated). Every GPU phase is timed between
    stream synchronisations. Returns the estimate, its standard errors and the figure of merit
    SE * sqrt(GPU seconds) of the plain and the control-variate estimates."""
    import torch
    import ttcf_inputs as I

    def sync_time(t0):
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    s = I.System(4)
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    ctx = T.Context(stream)
    r0, p0 = I.initial_state(s, seed)
    t0 = time.perf_counter()
    mid = ctx.ttcf_init_mother(sysd, r0, p0, n_equil=2000, n_melt=1000, t_melt=2.0)
    t_mother = sync_time(t0)
    n_rep = 256
    timings = {"mother_init_s": t_mother}

    def daughters(n_states, kick_seed, phase):
        t0 = time.perf_counter()
        per = n_states // n_rep
        ctx.ttcf_sample_states_replicated(mid, n_rep, seeded_kicks(n_rep, s.n, kick, kick_seed),
                                          decorrelate, per, 100)
        first = ctx.ttcf_spawn_daughters(mid, n_rep * per, 0, gd, nst)
        ctx.ttcf_step(nst)
        timings[phase + "_daughters_s"] = sync_time(t0)
        return first, 4 * n_rep * per

    # training set: three quarters train the network, one quarter calibrates beta(t)
    first, nd = daughters(train_states, seed * 1000 + 1, "train")
    n_fit = (3 * nd // 4) // 4 * 4
    n_out = nst
    ctx.ttcf_cv_init(n_out, _seeded_weights(n_out, seed))
    t0 = time.perf_counter()
    ctx.ttcf_cv_add_training(first, n_fit)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    order = np.stack([rng.permutation(n_fit).astype(np.int32) for _ in range(epochs)])
    loss = ctx.ttcf_cv_train(epochs, batch, lr, order)
    timings["training_s"] = sync_time(t0)
    t0 = time.perf_counter()
    ctx.ttcf_cv_attach(first + n_fit, nd - n_fit, T.TTCF_CV_CALIBRATE)
    ctx.ttcf_accumulate()  # training groups carry no control variate: they stay out of it
    beta = ctx.ttcf_cv_calibrate(nst + 1, gd)
    timings["calibration_s"] = sync_time(t0)
    # evaluation daughters with the control variate attached
    first, nd_eval = daughters(eval_states, seed * 1000 + 2, "eval")
    t0 = time.perf_counter()
    ctx.ttcf_cv_attach(first, nd_eval, T.TTCF_CV_ESTIMATE)
    timings["attach_s"] = sync_time(t0)
    t0 = time.perf_counter()
    ctx.ttcf_accumulate()
    timings["eval_accumulate_s"] = sync_time(t0)
    # mean term from independent branches
    t0 = time.perf_counter()
    n_mean = ctx.ttcf_cv_mean_term(mid, mean_replicas,
                                   seeded_kicks(mean_replicas, s.n, kick, seed * 1000 + 3),
                                   decorrelate, mean_rounds, mean_per_round, mean_between, gd)
    timings["mean_term_s"] = sync_time(t0)
    cm, cse, pm, pse, mu, mu_se, used = ctx.ttcf_cv_response(nst + 1, gd)
    ctx.close()
    t_plain = timings["eval_daughters_s"] + timings["eval_accumulate_s"]
    t_cv = t_plain + timings["train_daughters_s"] + timings["training_s"] + \
        timings["calibration_s"] + timings["attach_s"] + timings["mean_term_s"]
    se_cv = np.hypot(cse, mu_se)
    k = np.arange(1, nst + 1)
    gain = (pse[k] * np.sqrt(t_plain)) / (se_cv[k] * np.sqrt(t_cv))
    vr = (pse[k] / se_cv[k]) ** 2
    # with the fixed costs (training, calibration, mean term) spread over many more
    # evaluation daughters and the mean term's error made small: the per-daughter variance
    # ratio over the marginal cost ratio of a daughter with the control variate attached
    vr_pd = (pse[k] / cse[k]) ** 2
    marginal = (t_plain + timings["attach_s"]) / t_plain
    asym = np.sqrt(vr_pd / marginal)
    bias_bound = 2.0 * (pse + cse + mu_se)
    out = {
        "workload": f"WCA N={s.n}, rho={s.density}, T={s.temperature}, gamma_dot={gd}, "
                    f"{nst}-step daughters; {nd} training and {nd_eval} evaluation daughters; "
                    f"{n_mean} mean-term start states x 4 mappings; MLP 64-256-256-{n_out}, "
                    f"{epochs} epochs, batch {batch}, lr {lr}",
        "gain_at_t_end": float(gain[-1]),
        "gain_median": float(np.median(gain)),
        "gain_at_10_steps": float(gain[9]),
        "variance_ratio_at_steps": {str(j): float(vr[j - 1]) for j in (1, 10, 50, 100, nst)},
        "per_daughter_variance_ratio_at_steps": {str(j): float(vr_pd[j - 1])
                                                  for j in (1, 10, 50, 100, nst)},
        "marginal_cost_ratio": float(marginal),
        "asymptotic_gain_at_steps": {str(j): float(asym[j - 1]) for j in (1, 10, 50, 100, nst)},
        "fom_plain_t_end": float(pse[-1] * np.sqrt(t_plain)),
        "fom_cv_t_end": float(se_cv[-1] * np.sqrt(t_cv)),
        "gpu_s_plain": t_plain, "gpu_s_cv": t_cv,
        "ttcf_plain_t_end": float(pm[-1]), "se_plain_t_end": float(pse[-1]),
        "ttcf_cv_t_end": float(cm[-1]), "se_cv_t_end": float(se_cv[-1]),
        "bias_within_bound": bool(np.all(np.abs(cm - pm) <= bias_bound)),
        "train_loss_last_epoch": float(loss[-1]) if len(loss) else None,
        "n_states_eval": int(used), "timings_s": timings,
    }
    if verbose:
        out["series"] = {"beta": beta.tolist(), "plain": pm.tolist(), "plain_se": pse.tolist(), "cv": cm.tolist(),
                         "cv_se": se_cv.tolist(), "loss": loss.tolist()}
    return out


def cv_ceiling(T, stream, gd=1e-4, nst=200, n_states=256, siblings=8,
               scales=(1e-6, 1e-3, 1e-1), pos_scales=(1e-3, 1e-2), seed=6):
    """The most any start-state control variate can remove on the control-variate workload
    (N=256, rate 1e-4, 200-step daughters). Every start state gets `siblings` copies whose
    momenta carry a small zero-sum kick (scale x sqrt(T) per component), or whose positions
    are displaced (scale x the mean spacing rho^(-1/3) per component, momenta kept); their
    mapped daughters run 200 steps. G_n(t) = B(0) + int_0^t Omega(0) B(s) ds averaged over a state's
    four mappings (its contribution to Eq. TTCF). A one-way analysis of variance over states
    and siblings splits Var(G_n(t)) into the part the start state fixes, R^2 (stable under
    perturbations of that size), and the rest, which no function of the start state can
    predict at that resolution: a control variate of the start state reduces the standard
    error at most by 1 / sqrt(1 - R^2), with every cost left out."""
    import torch
    import ttcf_inputs as I
    s = I.System(4)
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    out = {"workload": f"{n_states} start states x {siblings} kicked siblings x 4 mappings x "
                       f"{nst} steps, N={s.n}, shear rate {gd}"}
    with T.Context(stream) as ctx:
        r0, p0 = I.initial_state(s, seed)
        mid = ctx.ttcf_init_mother(sysd, r0, p0, n_equil=2000, n_melt=1000, t_melt=2.0)
        ctx.ttcf_sample_states_replicated(mid, n_states,
                                          seeded_kicks(n_states, s.n, 0.05, seed * 1000 + 9),
                                          400, 1, 100)
        r, p = ctx.ttcf_export_states(mid, n_states)
        rng = np.random.Generator(np.random.PCG64(seed * 1000 + 10))
        spacing = s.density ** (-1.0 / 3.0)
        for kind, scale in [("kick", a) for a in scales] + [("shift", a) for a in pos_scales]:
            z = rng.standard_normal((n_states * siblings, 3, s.n))
            z -= z.mean(axis=2, keepdims=True)
            rs = np.repeat(r, siblings, axis=0)
            ps = np.repeat(p, siblings, axis=0)
            if kind == "kick":
                ps = ps + scale * np.sqrt(s.temperature) * z.reshape(n_states * siblings, -1)
            else:
                rs = np.mod(rs + scale * spacing * z.reshape(n_states * siblings, -1), s.box)
            ctx.ttcf_import_states(mid, rs, ps)
            first = ctx.ttcf_spawn_daughters(mid, n_states * siblings, 0, gd, nst)
            ctx.ttcf_step(nst)
            ser = ctx.ttcf_export_series(first, 4 * n_states * siblings, nst + 1)
            torch.cuda.synchronize()
            b = ser / s.volume                                   # P_xy(t) per daughter
            omega = -(gd / s.temperature) * ser[:, :1]           # Omega(0) = -(V/T) gd P_xy(0)
            f = omega * b
            integ = np.concatenate([np.zeros((len(f), 1)),
                                    np.cumsum(0.5 * (f[:, 1:] + f[:, :-1]) * s.dt, axis=1)], axis=1)
            g = (b[:, :1] + integ).reshape(n_states, siblings, 4, nst + 1).mean(axis=2)
            within = g.var(axis=1, ddof=1).mean(axis=0)          # per time point
            between = g.mean(axis=1).var(axis=0, ddof=1) - within / siblings
            r2 = np.clip(between / np.maximum(between + within, 1e-300), 0.0, 1.0)
            out[f"{kind}={scale:g}"] = {
                "r2_at_steps": {str(j): float(r2[j]) for j in (1, 10, 50, 100, nst)},
                "max_se_gain_at_steps": {str(j): float(1.0 / np.sqrt(max(1.0 - r2[j], 1e-12)))
                                         for j in (1, 10, 50, 100, nst)}}
            ctx.ttcf_accumulate()
    return out


def _seeded_weights(n_out: int, seed: int):
    """He-normal weights, zero biases, FP32 (numpy PCG64, seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    h, n_in = 256, 64
    parts = [rng.standard_normal((n_in, h)) * np.sqrt(2.0 / n_in), np.zeros(h),
             rng.standard_normal((h, h)) * np.sqrt(2.0 / h), np.zeros(h),
             rng.standard_normal((h, n_out)) * np.sqrt(1.0 / h), np.zeros(n_out)]
    return np.concatenate([a.ravel() for a in parts]).astype(np.float32)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-cells", type=int, default=8, help="fcc cells per edge (N = 4 n^3)")
    ap.add_argument("--states", type=int, default=1024)
    ap.add_argument("--daughter-steps", type=int, default=500)
    ap.add_argument("--precision", type=int, default=1, help="0 FP64 forces, 1 FP32 forces")
    ap.add_argument("--threads", type=int, default=0,
                    help="threads per workgroup (0: the library's choice)")
    ap.add_argument("--variant", type=int, default=0,
                    help="daughter kernel form: 0 auto, 1 cell list, 2 neighbour list")
    ap.add_argument("--skin", type=float, default=0.0, help="neighbour-list skin (0: default)")
    ap.add_argument("--kmax", type=int, default=0, help="neighbour-list capacity (0: default)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 to skip)")
    ap.add_argument("--fp64-check", type=int, default=1,
                    help="1: rerun the batch's start states with FP64 forces at every shear rate "
                         "and report the FP32-force error of each response")
    ap.add_argument("--thermostats", type=int, default=1,
                    help="1: also compare isokinetic and Nose-Hoover daughters on the same states")
    ap.add_argument("--observables", type=int, default=1,
                    help="1: also measure daughters that record the extra bulk observables")
    ap.add_argument("--mixed", type=int, default=1,
                    help="1: also measure mixed-flow daughters on the same start states")
    ap.add_argument("--elongation", type=int, default=1,
                    help="1: also measure planar-elongation daughters on the same start states")
    ap.add_argument("--colour", type=int, default=1,
                    help="1: also measure colour-field daughters on the same start states")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: also measure whole cycles replayed from a captured graph")
    ap.add_argument("--uneven", type=int, default=1,
                    help="1: also measure the mixed-size batch (report under 'uneven')")
    ap.add_argument("--channel", type=int, default=1,
                    help="1: also measure the confined-channel workload (report under 'channel')")
    ap.add_argument("--cv", type=int, default=1,
                    help="1: also measure the learned control variate (N=256, shear rate 1e-4 "
                         "workload) and report it under 'cv'")
    ap.add_argument("--pipeline", type=int, default=1,
                    help="1: two contexts take the headline batches in turn, one's host work "
                         "overlapping the other's kernel; 0: one context")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a kernel of known "
                         "traffic, used to calibrate the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the daughter path shards by start state, and "
              "it measures one GPU's share.", file=sys.stderr)
        sys.exit(2)

    import torch

    import ttcf_inputs as I
    from paper_2312_02990_amd import ttcf as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        nel = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    T.use_torch_allocator()
    stream = T.current_stream()
    s = I.System(args.n_cells)
    sysd = T.make_system(s.n, s.box, s.temperature, s.dt, precision=args.precision,
                         block_threads=args.threads)
    r0, p0 = I.initial_state(s, 2)
    ctx = T.Context(stream)
    t0 = time.perf_counter()
    mid = ctx.ttcf_init_mother(sysd, r0, p0, n_equil=2000, n_melt=1000, t_melt=2.0)
    ctx.ttcf_set_step_shape(args.variant, args.threads, args.skin, args.kmax)
    ctx.ttcf_record_mother(mid, 100 * args.states)
    ctx.ttcf_sample_states(mid, args.states, 100)
    torch.cuda.synchronize()
    mother_s = time.perf_counter() - t0
    # the sampling interval against the correlation time of the mother's V*P_xy
    acf_vals, acf_first, acf_tau = ctx.ttcf_mother_acf(mid, 400, 0.05)
    mother_acf = {"steps_between": 100, "first_lag_below_0.05": acf_first,
                  "integrated_correlation_steps": acf_tau,
                  "acf_at_steps_between": float(acf_vals[100])}
    mother_steps = 3000 + 100 * args.states

    nst = args.daughter_steps
    n_d = 4 * args.states
    # per shear rate: groups expected and healthy so far (a rate's response covers every
    # batch run at it), and the latest response
    expected, healthy, responses = {}, {}, {}

    # With --pipeline 1, two contexts on two streams take the batches in turn (batch i in
    # context i mod 2, so each shear rate's groups stay in one context, the rates cycling
    # through four values): one context's host bookkeeping (the accumulation and response of
    # its last batch, then its next spawn) runs while the other's kernel does. The step
    # kernels are chained by events, so they never share the GPU; the per-launch kernel times
    # stay those of a kernel alone.
    # (both on streams of their own: work on the legacy default stream would wait for every
    # other stream's, and theirs for it)
    ctxs = [(ctx, mid, torch.cuda.current_stream())]
    if args.pipeline:
        import ctypes
        r_st, p_st = ctx.ttcf_export_states(mid, args.states)
        ctxs = []
        for _ in range(2):
            sk = torch.cuda.Stream()
            ck = T.Context(ctypes.c_void_p(sk.cuda_stream))
            mk = ck.ttcf_init_mother(sysd, r_st[0], p_st[0], n_equil=0)
            ck.ttcf_set_step_shape(args.variant, args.threads, args.skin, args.kmax)
            ck.ttcf_import_states(mk, r_st, p_st)
            ctxs.append((ck, mk, sk))
        del r_st, p_st

    def spawn_step(i, after):
        c, m, st = ctxs[i % len(ctxs)]
        gd = GAMMAS[i % len(GAMMAS)]
        c.ttcf_spawn_daughters(m, args.states, 0, gd, nst)
        if after is not None:
            st.wait_event(after)
        c.ttcf_step(nst)
        done = torch.cuda.Event()
        done.record(st)
        return gd, done

    def finish(i, gd):
        c = ctxs[i % len(ctxs)][0]
        c.ttcf_accumulate()
        res = c.ttcf_response(nst + 1, gd)
        new = res[4] - healthy.get(gd, 0)  # healthy groups of this batch
        expected[gd] = expected.get(gd, 0) + args.states
        healthy[gd] = res[4]
        responses[gd] = res
        return new

    def run_batches(first, count):
        """Batches first .. first + count - 1; returns their healthy groups."""
        total, pending, after = 0, None, None
        for i in range(first, first + count):
            if len(ctxs) == 1:
                gd, _ = spawn_step(i, None)
                total += finish(i, gd)
                continue
            gd, after = spawn_step(i, after)
            if pending is not None:
                total += finish(*pending)
            pending = (i, gd)
        if pending is not None:
            total += finish(*pending)
        return total

    run_batches(0, args.warmup)
    for c, _, _ in ctxs:
        c.ttcf_step_timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    healthy_timed = run_batches(args.warmup, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = 0.0, 0
    for c, _, _ in ctxs:
        km, kl = c.ttcf_step_timing(reset=True)
        kern_ms += km
        launches += kl

    start_states = ctx.ttcf_export_states(mid, args.states) if args.cpu_budget > 0 else None
    progress("headline")
    precision = None
    if args.precision == 1 and args.fp64_check:
        precision = precision_statement(T, ctx, mid, sysd, s, args.states, nst, stream)
    progress("precision")
    green_kubo = None
    try:
        green_kubo = green_kubo_leg(T, ctx, mid, s, 100 * args.states, nst,
                                    resp_ctx=ctxs[GAMMAS.index(1e-4) % len(ctxs)][0])
    except Exception as e:  # the headline line is printed whatever happens here
        green_kubo = {"error": repr(e)}
    for c, _, _ in ctxs:
        if c is not ctx:
            c.close()
    thermostats = None
    progress("green-kubo")
    if args.thermostats:
        try:
            thermostats = thermostat_leg(T, stream, ctx, mid, s, args.states, nst)
        except Exception as e:  # the headline line is printed whatever happens here
            thermostats = {"error": repr(e)}
    observables = None
    progress("thermostats")
    if args.observables:
        try:
            observables = observables_leg(T, stream, ctx, mid, s, args.states, nst)
        except Exception as e:  # the headline line is printed whatever happens here
            observables = {"error": repr(e)}
    elongation = None
    progress("observables")
    if args.elongation:
        try:
            elongation = elongation_leg(T, stream, ctx, mid, s, args.states, nst)
        except Exception as e:  # the headline line is printed whatever happens here
            elongation = {"error": repr(e)}
    mixed = None
    progress("elongation")
    if args.mixed:
        try:
            mixed = mixed_leg(T, stream, ctx, mid, s, args.states, nst)
        except Exception as e:  # the headline line is printed whatever happens here
            mixed = {"error": repr(e)}
    colour = None
    progress("mixed")
    if args.colour:
        try:
            colour = colour_leg(T, stream, ctx, mid, s, args.states, nst)
        except Exception as e:  # the headline line is printed whatever happens here
            colour = {"error": repr(e)}
    ctx.close()

    atom_steps = n_d * s.n * nst
    # only the daughters of healthy groups count (a group whose list overflowed stops early)
    value = 4 * healthy_timed * s.n * nst / wall
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    achieved = BYTES_PER_ATOM_STEP * atom_steps / avg_launch_s / 1e9
    traffic = measured_traffic()
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "daughter atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair forces / f64 integration and sums" if args.precision
                 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batched bulk WCA: N={s.n}, rho={s.density}, T={s.temperature}, "
                        f"dt={s.dt}; {args.states} start states x 4 mappings = {n_d} daughters "
                        f"x {nst} steps per batch, one persistent launch; shear rate cycling "
                        f"{list(GAMMAS)}",
            "n_atoms": s.n, "daughters": n_d, "daughter_steps": nst,
            "parallelism": "one GPU",
            "host_pipeline": (f"{len(ctxs)} contexts take the batches in turn; step kernels "
                              "chained by events, never concurrent") if len(ctxs) > 1
                             else "one context",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_daughters_pairs (persistent pair-list daughter step kernel)",
            "kernel_ms_per_launch": 1e3 * avg_launch_s,
            "algorithmic_bytes_per_launch": BYTES_PER_ATOM_STEP * atom_steps,
            "valu": measured_valu(),
        },
        "kernel_atom_steps_per_s": atom_steps / avg_launch_s,
        "mother_s": mother_s,
        "mother_acf": mother_acf,
        "mother_atom_steps_per_s": mother_steps * s.n / mother_s,
        "healthy_groups_timed": {"healthy": int(healthy_timed),
                                 "expected": int(args.states * args.steps),
                                 "all_healthy": int(healthy_timed) == args.states * args.steps},
        "per_rate": per_rate_statement(responses, expected, nst, s.dt),
    }
    if precision is not None:
        line["precision"] = precision
    if green_kubo is not None:
        line["green_kubo"] = green_kubo
    if thermostats is not None:
        line["thermostats"] = thermostats
    if observables is not None:
        line["observables"] = observables
    if colour is not None:
        line["colour"] = colour
    if elongation is not None:
        line["elongation"] = elongation
    if mixed is not None:
        line["mixed"] = mixed
    progress("colour")
    if args.graph:
        try:
            line["graph"] = graph_leg(T, stream)
        except Exception as e:  # the headline line is printed whatever happens here
            line["graph"] = {"error": repr(e)}
    progress("graph")
    if args.uneven:
        try:
            line["uneven"] = uneven_leg(T, stream)
        except Exception as e:  # the headline line is printed whatever happens here
            line["uneven"] = {"error": repr(e)}
    progress("uneven")
    if args.channel:
        try:
            line["channel"] = channel_leg(T, stream)
        except Exception as e:  # the headline line is printed whatever happens here
            line["channel"] = {"error": repr(e)}
    progress("channel")
    if args.cv:
        try:
            line["cv"] = cv_leg(T, stream)
        except Exception as e:  # the headline line is printed whatever happens here
            line["cv"] = {"error": repr(e)}
        try:
            line["cv"]["ceiling"] = cv_ceiling(T, stream)
        except Exception as e:  # the headline line is printed whatever happens here
            line["cv"]["ceiling"] = {"error": repr(e)}
    progress("cv")
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(args.n_cells, nst, args.cpu_budget, start_states)
        try:
            line["cpu_baseline_other_configs"] = cpu_baseline_configs()
        except Exception as e:  # the headline line is printed whatever happens here
            line["cpu_baseline_other_configs"] = {"error": repr(e)}
    progress("cpu baseline")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

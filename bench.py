"""Throughput benchmark: env-steps/s at NCP residual 1e-6 on one MI355X.

Workload (squeeze_blocks): 1024 environments, each a 10x10x10-hex block (1331
vertices, 6000 tets, E ~ U(5e4, 5e5) Pa, nu ~ U(0.30, 0.45), mu ~ U(0.3,
0.8)) resting on the ground and squeezed by two kinematic box fingers closing
at 2 cm/s, about 220 contacts per env, h = 1/60 s, 20 local-global iterations
per step, FP32, every contact solve run to the NCP tolerance.  Inputs are
seeded and synthetic and stand in for the paper's garment and towel scenes.

A step is one pass of the whole hot path over all environments (detection,
prediction, K x (projection, assembly, global apply, contact solve, position
update), finalisation).  The state is resident in HBM before the timed region:
W warm-up steps (--warmup), then K timed steps (--steps) bracketed by device
synchronisation, so the timed window is steps W .. W+K-1 of the squeeze.

Arms, each on a fresh batch over the same steps:
  plain            A1: previous-step warm start, one launch per phase, one
                   stream, no graph; every launch timed with HIP events.
  batched          A2: the local-global loop as one launch per step with one
                   workgroup per env (k_lg_fused), one stream; previous-step start.
  batched_learned  A3 (value): as batched, with the learned warm start.  Its
                   network is trained first, on the GPU, from a recorded
                   zero-start rollout with seeds disjoint from the timed
                   workload (4,000,000 pairs); recording and training are
                   reported separately and excluded from the timed region.
                   The k_lg_fused launches of this arm's timed steps are timed
                   with HIP events on the batch's stream: the roofline.
  batched_groups   the learned configuration on 3 env groups with their own
                   streams and HIP graphs (context: the same kernels, one
                   group's tail overlapping the others' work).
  cold_starts      plain vs learned start when every env's multiplier history
                   is dropped every 5 steps (as episode resets do), both at
                   the same tolerance: Newton iterations and env-steps/s.
  uneven_batched   a second workload: 4096 envs of the uneven mixed recipe
                   (cloth sheets and tet blocks, moving obstacles), 3 groups.
  fold_sweep       Table II-style throughput: ms/step of the cloth-folding stand-in
                   (cloth_fold: 64 x 64 sheet on a mu = 1 table, two grippers folding
                   the near corners over, h = 0.01, FP32, lightweight metric from
                   global memory, HIP graph) at 1, 8, 32, 64, 128 and 256 envs, with
                   the paper's budget (5 local-global iterations x 10 updates) and
                   its low-iteration ablation (2 x 2); the paper's own RTX 4090
                   figures ride along as context.
  depth_render     batched depth ray casting (depth, instance ids): a draped
                   181 x 181 towel stand-in (32,761 vertices, the size of the
                   paper's towel-folding scene) over a table, per-env seeded folds,
                   one top-down camera per env, at 1, 8, 32, 64 and 128 envs and
                   at 640 x 480 and 128 x 128 pixels: ms per frame (hierarchy refit
                   + render), with the paper's own figures as context.
  uneven_full      (opt-in, not in the default set) the uneven recipe at its
                   configured sizes: sheets up to 48 x 48 and tet blocks up to
                   8000 vertices, K = 10, FP32, lightweight metric from global
                   memory with a budget of 10 updates (sheets lying on the ground
                   exceed what the exact solve holds in LDS); create time (host
                   precompute of the explicit inverses) reported separately; the
                   largest sheet and the largest block checked against the oracle's
                   lightweight step from a history reset.
  slab_press       (opt-in) the large-scene recipe: 64 envs of a 102,010-vertex,
                   540,000-tet slab pressed by two pads (at most 20k contacts), FP32,
                   lightweight metric from global memory, K = 10, budget 10, HIP
                   graph; the envs are copies and share one explicit inverse
                   (41.6 GB); create time and the HBM footprint reported; env 0
                   checked against the oracle's lightweight step from a history
                   reset.
  squeeze_horizon  (opt-in) the squeeze's whole 500-step horizon from its first step
                   in the batched configuration (the local-global loop as one launch
                   per step, one stream, previous-step warm start, every contact solve
                   to 1e-6 m): env-steps/s over all 500 steps, ms per step in blocks
                   of 50 steps (closing, then holding), residual and Newton counts.
  contact_metric   the exact contact-space metric Z = h^2 J A^-1 H^T + E (Eq. 7)
                   against the inertia-only Z~ (Eq. 10), on the dropped cube
                   (FP64, 1 env, 120 steps) and on the squeeze workload from the
                   state at the start of the timed window: updates per local-
                   global iteration, ms/step and the residual reached, with Z~
                   both run to the tolerance and held to the paper's budget of
                   10 updates per local-global iteration.

After each arm's timed window one more step of sampled envs is checked against
the FP64 oracle from the GPU's own state (oracle_error: max absolute and
relative position error, and the NCP residual the oracle computes from the GPU's
positions and multipliers).

Roofline (HBM) of the dominant kernel k_lg_fused in the reported arm: the
algorithmic bytes of the path per env-step (the per-sweep formulas: detection
24 n_v + 64 n_c; per local-global iteration projection + assembly 56 n_tet +
36 n_v and one global apply 8 nnz(S) + 36 n_v with nnz(S) = n_v (n_v + 1) / 2;
108 n_c per Newton iteration; finalisation 48 n_v), summed over envs with the
window's measured Newton iterations, divided by the average event-timed launch
duration.  Detection and finalisation run in their own small kernels; their
bytes (under 0.1%) stay in the numerator.  Bytes this implementation moves
beyond the formula (vertex forces through HBM, incidence lists, the position
update's second read of the contact rows of the inverse) are reported in
overhead_bytes_per_launch and count against the fraction.  `traffic` comes
from a committed counter summary when it was taken on the same kernel source.

--profile-window brackets the reported arm's timed steps with
roctxProfilerResume / roctxProfilerPause (the rest of the run is paused), so
that `rocprofv3 --selected-regions` traces exactly the timed window.

cpu_baseline: the FP64 oracle on the host on a bounded sample of the same
workload: sampled envs from the GPU's state at the start of the timed window,
the window's first steps, at 1 thread and on all cores given to this process.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/sec at NCP residual 1e-6: plain vs batched+learned warm-start, 1 GPU"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
K_FUSED_BIT = 1 << 9          # kernel class of k_lg_fused in flash_kernel_name order
ALL_ARMS = ("plain", "batched", "batched_learned", "batched_groups", "cold_starts", "uneven_batched",
            "contact_metric", "fold_sweep", "depth_render")
OPT_IN_ARMS = ("uneven_full", "slab_press", "squeeze_horizon")
RENDER_ENVS = (1, 8, 32, 64, 128)
# the paper's depth-rendering overhead table (towel-folding scene, ms per frame): context only
PAPER_RENDER_MS = {1: 0.75, 8: 2.23, 32: 7.20, 64: 14.18, 128: 27.31}
FOLD_ENVS = (1, 8, 32, 64, 128, 256)
# Table II of the paper (FLASH row, ms/step on one RTX 4090, T-shirt dual-sleeve folding): context only
PAPER_TABLE_II = {1: 5.68, 8: 9.67, 32: 24.79, 64: 50.43, 128: 90.41, 256: 185.10}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- bytes

def path_bytes(envs, contacts, K, newton_per_env_step):
    """Algorithmic bytes of one step of the listed envs (FP32 values, int32 indices)."""
    tot = 0.0
    for env, c, nw in zip(envs, contacts, newton_per_env_step):
        n, T = float(env.n_vertices), float(env.n_elements)
        b_detect = 24 * n + 64 * c
        b_proj = 56 * T + 36 * n
        b_apply = 8 * n * (n + 1) / 2 + 36 * n
        b_contact = 108 * c
        b_fin = 48 * n
        tot += b_detect + K * (b_proj + b_apply) + nw * b_contact + b_fin
    return tot


def overhead_bytes(envs, contacts, K):
    """Bytes beyond the formula per step: vertex forces written and read back (96 per tet), incidence
    slots (16 per tet) and the position update's read of the contact rows of the inverse (4 n_v n_c)."""
    tot = 0.0
    for env, c in zip(envs, contacts):
        n, T = float(env.n_vertices), float(env.n_elements)
        tot += K * (112 * T + 4 * n * c)
    return tot


def apply_bytes_per_launch(nv):
    """Bytes of one batched global-apply launch as this implementation stores the inverse (full n x n)."""
    nv = np.asarray(nv, dtype=np.float64)
    return float(np.sum(4.0 * nv * nv + 2 * 12.0 * nv))


def source_hash(*paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:12]


def kernel_source_hash(path, *names):
    """sha256 (12 hex digits) of the source text of the named templates."""
    import hashlib
    src = open(path).read()
    parts = []
    for name in names:
        i = src.index(f"{name}(")
        i = src.rfind("template <", 0, i)
        j = src.index("\n}\n", i)
        parts.append(src[i:j + 3])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:12]


def committed_traffic(path, src_hash):
    """HBM bytes per launch from a committed counter summary, if it was taken on this kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "kernel_source_sha256")):
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != src_hash or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


# ----------------------------------------------------------------------------- oracle legs

def _warm_imports(_=None):
    """Imports the oracle's modules in a worker process (kept out of the timed oracle steps)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import threadpoolctl  # noqa: F401
    from oracle import flash_oracle  # noqa: F401
    return os.getpid()


def _oracle_job(env, x, v, obs, params, n_steps, threads_limit):
    """FP64 oracle steps of one env from a given state (worker process, precompute untimed); returns
    (seconds, last residual)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits
    from oracle import flash_oracle as O
    with threadpool_limits(limits=threads_limit):
        oe = O.precompute(env, params.h)
        t0 = time.time()
        r = None
        for _ in range(n_steps):
            r = O.step(oe, x, v, obs, params)
            x, v, obs = r.x, r.v, r.obstacles
        return time.time() - t0, (r.residual if r is not None else 0.0)


def _oracle_check(env, x0, v0, obs, params, x1, lam, verts, obsi):
    """One oracle step from (x0, v0); error of the GPU end state x1 and the oracle residual of the GPU's
    positions and multipliers."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits
    from oracle import flash_oracle as O
    with threadpool_limits(limits=1):
        oe = O.precompute(env, params.h)
        ref = O.step(oe, x0, v0, obs, params, tol=1e-12)
        L = float(np.linalg.norm(env.rest_x.max(0) - env.rest_x.min(0)))
        err = float(np.abs(x1 - ref.x).max())
        scale = max(float(np.abs(ref.x).max()), L)
        same = list(zip(verts, obsi)) == list(zip(ref.contacts.vertex.tolist(), ref.contacts.obstacle.tolist()))
        r = O.contact_residual(oe, x0, x1, ref.contacts, lam, params.h) if same else float("inf")
        return err, err / scale, same, r


def spawn_pool(n):
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(n)


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


# ----------------------------------------------------------------------------- GPU legs

def train_warm_start(F, scenes, torch, pairs=4_000_000, n_envs=320, epochs=6, seed=1):
    """Records cold-start training pairs (zero warm start: every contact of every step lacks a previous
    multiplier) from a squeeze rollout with seeds disjoint from the timed workload until `pairs` rows are
    held, and fits the warm-start network on exactly `pairs` of them on the GPU."""
    t0 = time.time()
    sc = scenes.squeeze_blocks(n_envs, seed=seed)
    b = F.from_scene(sc, warm_start=F.FLASH_WS_ZERO)
    cap = pairs + n_envs * 320
    fd = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
    ld = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    b.ws_record(True)
    n, steps = 0, 0
    while n < pairs:
        b.step(1)
        n = b.ws_collect(fd, ld, cap, n)
        steps += 1
    b.close()
    t_rec = time.time() - t0
    m = F.Mlp(max_rows=65536, seed=seed)
    m.fit_norm(fd, ld, pairs)
    t1 = time.time()
    losses = []
    for ep in range(epochs):
        lr = 1e-3 if ep < epochs - 2 else 3e-4
        losses += m.train(fd, ld, pairs, epochs=1, batch=4096, lr=lr, seed=ep).tolist()
    torch.cuda.synchronize()
    t_train = time.time() - t1
    info = {"pairs": int(pairs), "recorded": int(n), "record_s": round(t_rec, 1), "train_s": round(t_train, 2),
            "epochs": epochs, "batch": 4096, "epoch_loss": [round(x, 5) for x in losses],
            "train_rows_per_s": round(pairs * epochs / t_train),
            "source": f"squeeze_blocks({n_envs}, seed={seed}), {steps} steps, zero warm start"}
    w, nm = m.params_bf16(), m.norm()
    del fd, ld
    m.close()
    return w, nm, info


def mlp_roofline(F, torch, rows=1 << 22, reps=5):
    """Fused bf16 MFMA forward pass over `rows` feature rows, timed with HIP events on the stream it
    runs on: algorithmic 70,400 FLOP per row against the dense bf16 peak."""
    st = torch.cuda.current_stream()
    m = F.Mlp(max_rows=4096, seed=0, stream=st.cuda_stream)
    x = torch.randn((rows, 16), dtype=torch.float32, device="cuda")
    y = torch.empty((rows, 3), dtype=torch.float32, device="cuda")
    m.forward(x, rows, y)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        m.forward(x, rows, y)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    tflops = 70400.0 * rows / (ms * 1e-3) / 1e12
    m.close()
    return {"bound": "mfma", "kernel": "k_mlp_fused (16-128-128-128-3 forward, v_mfma_f32_32x32x16_bf16)",
            "achieved": round(tflops, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None, "rows_per_launch": rows,
            "flop_per_row": 70400, "avg_launch_ms": round(ms, 4)}


class Roctx:
    """roctxProfilerPause / roctxProfilerResume (no-ops when the library is absent)."""

    def __init__(self, on):
        self.lib = None
        if on:
            for name in ("librocprofiler-sdk-roctx.so", "/opt/rocm/lib/librocprofiler-sdk-roctx.so"):
                try:
                    lib = ctypes.CDLL(name)
                    lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]
                    lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
                    self.lib = lib
                    break
                except (OSError, AttributeError):
                    continue
            if self.lib is None:
                log("roctx library not found: --profile-window has no effect")

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)


def run_arm(F, sc, args, *, warm_start, ws=None, use_graph=False, groups=0, fused=False, timing=0,
            reset_every=0, roctx=None, sample=(), check=True, capture=0):
    """Fresh batch of the workload: W warm-up steps, then K timed steps (synchronised both sides).
    timing: kernel classes bracketed by HIP events in the timed steps; reset_every: drop every env's
    multiplier history every that many timed steps (device-side state round trip).  Returns a result
    dict and the oracle check jobs of the sampled envs (one extra, untimed step)."""
    import torch
    t0 = time.time()
    b = F.from_scene(sc, use_graph=use_graph, warm_start=warm_start, stream_groups=groups, fused_lg=fused)
    t_create = time.time() - t0
    if ws is not None:
        b.ws_load(*ws)
    b.step(args.warmup)
    b.synchronize()
    start_state = None
    if capture:
        # the state at the start of the timed window (read before the timed region starts)
        x0, v0 = b.get_state()
        start_state = (b.split(x0)[:capture], b.split(v0)[:capture], [b.get_obstacles(e) for e in range(capture)])
    b.residual_history(reset=True)
    b.ws_history(reset=True)
    xs = vs = None
    if reset_every:
        nv = sum(e.n_vertices for e in sc.envs)
        xs = torch.empty((3, nv), dtype=torch.float32, device="cuda")
        vs = torch.empty((3, nv), dtype=torch.float32, device="cuda")
    if timing:
        b.set_kernel_timing(timing)
    torch.cuda.synchronize()
    if roctx is not None:
        roctx.resume()
    t1 = time.perf_counter()
    if reset_every:
        done = 0
        while done < args.steps:
            n = min(reset_every, args.steps - done)
            b.get_state_device(xs, vs)
            b.set_state_device(xs, vs)       # same state, no multiplier history
            b.step(n)
            done += n
    else:
        b.step(args.steps)
    b.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    if roctx is not None:
        roctx.pause()
    kt = b.kernel_times() if timing else None
    b.set_kernel_timing(0)
    mx, failed, newton, env_steps = b.residual_history(reset=True, full=True)
    started, restarted = b.ws_history(reset=True)
    stats = b.stats()
    dropped = sum(1 for s_ in stats if s_["flags"] & 4)
    assert dropped == 0, f"{dropped} envs dropped contacts beyond the capacity in the timed window"
    res = {"env_steps_per_s": round(len(sc.envs) * args.steps / dt, 2), "ms_per_step": round(1000 * dt / args.steps, 3),
           "max_residual": mx, "env_steps_failed": int(failed), "newton_per_env_step": round(newton / max(env_steps, 1), 3),
           "create_s": round(t_create, 1)}
    if warm_start == F.FLASH_WS_LEARNED:
        res["env_steps_started_from_prediction"] = int(started)
        res["env_steps_restarted_from_plain_start"] = int(restarted)
    extra = {"batch": b, "dt": dt, "kt": kt, "stats": stats, "newton_per_env_step": newton / max(env_steps, 1),
             "start_state": start_state}
    jobs = []
    if check and sample:
        x0, v0 = b.get_state()
        obs = {e: b.get_obstacles(e) for e in sample}
        b.step(1)
        x1, _ = b.get_state()
        xs0, vs0, xs1 = b.split(x0), b.split(v0), b.split(x1)
        for e in sample:
            c = b.contacts(e)
            jobs.append((sc.envs[e], xs0[e], vs0[e], obs[e], sc.params, xs1[e], c["lambda"],
                         c["vertex"].tolist(), c["obstacle"].tolist()))
    return res, extra, jobs


def _timed_metric_run(F, sc, prec, metric, cap, steps, blob=None, warm=0):
    """One solver variant from a state (a checkpoint, or `warm` steps from the scene's start):
    steps timed with device synchronisation on both sides."""
    sc.params.max_inner_iterations = cap
    b = F.from_scene(sc, precision=prec, contact_metric=metric, fused_lg=True)
    if blob is not None:
        b.load_checkpoint(blob)
    elif warm:
        b.step(warm)
    b.synchronize()
    b.residual_history(reset=True)
    t = time.perf_counter()
    b.step(steps)
    b.synchronize()
    dt = (time.perf_counter() - t) / steps
    mx, over, newton, st = b.residual_history(reset=True, full=True)
    b.close()
    return {"ms_per_step": round(1e3 * dt, 3), "env_steps_per_s": round(len(sc.envs) / dt, 1),
            "updates_per_lg_iteration": round(newton / max(st, 1) / sc.params.lg_iterations, 3),
            "max_residual_m": float(f"{mx:.3e}"), "env_steps_above_tol": int(over), "env_steps": int(st),
            "steps_timed": steps}


def metric_compare(F, scenes, args):
    """Exact metric against the inertia-only metric (to the tolerance, and at a budget of 10)."""
    out = {}
    variants = (("exact", 0, 50), ("lightweight_to_tol", 1, 20000), ("lightweight_budget_10", 1, 10))
    c1 = {}
    for name, metric, cap in variants:
        c1[name] = _timed_metric_run(F, scenes.drop_cube(seed=0), F.FLASH_FP64, metric, cap, 120)
    out["C1_drop_cube_fp64"] = c1
    sc = scenes.squeeze_blocks(args.envs, seed=0)
    b = F.from_scene(sc, fused_lg=True)
    b.step(args.warmup)
    blob = b.save_checkpoint()
    b.close()
    c2 = {}
    for name, metric, cap in variants:
        n = 2 if name == "lightweight_to_tol" else args.steps
        c2[name] = _timed_metric_run(F, scenes.squeeze_blocks(args.envs, seed=0), F.FLASH_FP32, metric, cap, n,
                                     blob=blob)
    out[f"C2_squeeze_blocks_{args.envs}_fp32_from_step_{args.warmup}"] = c2
    out["note"] = ("every variant solves each local-global iteration's contact problem to the same inner "
                   "tolerance (exact and lightweight_to_tol) or stops at 10 updates (lightweight_budget_10); "
                   "updates are semismooth Newton iterations for the exact metric, block updates for Z~")
    return out


def fold_sweep(F, scenes, args):
    """ms/step of the folding stand-in against the env count (Table II's layout)."""
    n = args.fold_side
    out = {"workload": f"cloth_fold: {n}x{n} sheet ({n * n} vertices, {2 * (n - 1) ** 2} triangles) on a "
                       f"mu = 1 table, two grippers folding the near corners, h = 0.01 s, FP32, lightweight "
                       f"metric from global memory, HIP graph; window: steps {args.fold_warmup}.."
                       f"{args.fold_warmup + args.fold_steps - 1} of the fold",
           "rows": {}}
    for name, (K, N) in (("lg5_linear10", (5, 10)), ("lg2_linear2", (2, 2))):
        row = {}
        for ne in args.fold_envs:
            sc = scenes.cloth_fold(ne, n=n, lg_iterations=K, inner_iterations=N)
            b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, max_contacts=n * n + 8, use_graph=True)
            b.step(args.fold_warmup)
            b.synchronize()
            b.residual_history(reset=True)
            t = time.perf_counter()
            b.step(args.fold_steps)
            b.synchronize()
            dt = (time.perf_counter() - t) / args.fold_steps
            mx, over, newton, st = b.residual_history(reset=True, full=True)
            cts = [s_["contacts"] for s_ in b.stats()]
            b.close()
            row[str(ne)] = {"ms_per_step": round(1e3 * dt, 3), "env_steps_per_s": round(ne / dt, 1),
                            "updates_per_lg_iteration": round(newton / max(st, 1) / K, 2),
                            "max_residual_m": float(f"{mx:.3e}"), "contacts_per_env": int(np.mean(cts))}
            log(f"fold sweep {name}: {ne} envs {row[str(ne)]['ms_per_step']} ms/step")
        out["rows"][name] = row
    out["paper_table_ii_ms_per_step_rtx4090"] = {str(k): v for k, v in PAPER_TABLE_II.items()}
    out["note"] = ("the paper's scene is a T-shirt of unstated size; this stand-in's mesh is stated above; "
                   "the paper's figures are another machine's and another mesh's (context, not a target)")
    return out


def towel_positions(rest, n, seed):
    """A draped towel stand-in: the flat sheet lifted into seeded folds 0-6 cm above the table."""
    rng = np.random.default_rng(seed)
    x = rest.copy()
    k = rng.uniform(6.0, 14.0, size=2)
    ph = rng.uniform(0.0, 2 * np.pi, size=2)
    x[:, 1] = 0.03 + 0.03 * np.sin(k[0] * rest[:, 0] + ph[0]) * np.cos(k[1] * rest[:, 2] + ph[1])
    return x


def depth_render(F, scenes, torch, args):
    """ms per frame of the batched renderer against the env count (the paper's rendering table)."""
    n = 181
    rest, tris = scenes.cloth_grid(n, 0.6, (-0.3, -0.3), 0.0)
    env = scenes.EnvDesc(scenes.TRI, rest, tris, density=1000.0, thickness=1e-3, young=3e4, poisson=0.4,
                         bending=0.2, mu=1.0)
    down = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    out = {"workload": f"towel stand-in: {n}x{n} sheet ({n * n} vertices, {2 * (n - 1) ** 2} triangles) in seeded "
                       f"folds over a table plane, one top-down camera per env at 0.9 m (fx = fy = 0.78 x width); "
                       f"outputs depth and instance ids; positions resident on the GPU; refit + render per frame",
           "rows": {}}
    for (W, H) in ((640, 480), (128, 128)):
        row = {}
        cam = {"position": np.array([0.0, 0.9, 0.0]), "rot": down, "fx": 0.78 * W, "fy": 0.78 * W,
               "cx": W / 2.0, "cy": H / 2.0}
        for ne in RENDER_ENVS:
            xs = np.concatenate([towel_positions(rest, n, s) for s in range(ne)]).T.copy()
            x = torch.tensor(xs, dtype=torch.float32, device="cuda")
            R = F.Renderer([env] * ne)
            obs = [[scenes.ground()]] * ne
            for _ in range(2):
                R.render(x, [cam] * ne, W, H, obstacles=obs)
            reps = 10
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                o = R.render(x, [cam] * ne, W, H, obstacles=obs)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            cover = float((o["instance"] == 0).float().mean().item())
            R.close()
            row[str(ne)] = {"ms_per_frame": round(1e3 * dt, 3), "mrays_per_s": round(ne * W * H / dt / 1e6, 1),
                            "towel_pixels_frac": round(cover, 3)}
            log(f"depth render {W}x{H}: {ne} envs {row[str(ne)]['ms_per_frame']} ms/frame")
            del x
        out["rows"][f"{W}x{H}"] = row
    out["paper_ms_per_frame"] = {str(k): v for k, v in PAPER_RENDER_MS.items()}
    out["note"] = ("the paper does not state its image size; its figures (another machine, its own ray-casting "
                   "backend) are context, not a target")
    return out


def uneven_full(F, scenes, args):
    """The uneven recipe at its configured sizes, lightweight metric from global memory."""
    from oracle import flash_oracle as O     # the oracle check of two sampled envs (test infrastructure)
    ne = args.uneven_full_envs
    su = scenes.uneven_batch(ne, seed=7, max_tet_vertices=8000, max_cloth_side=48, lg_iterations=10)
    su.params.max_inner_iterations = 10
    nv = [e.n_vertices for e in su.envs]
    # created in chunks of at most 1024 envs (each on a stream of its own, stepped together as
    # stream groups would be) so that the host precompute reports progress
    chunk = 1024
    t0 = time.perf_counter()
    parts = []
    for c0 in range(0, ne, chunk):
        c1 = min(ne, c0 + chunk)
        sub = scenes.Scene(su.envs[c0:c1], su.x0[c0:c1], su.v0[c0:c1], su.obstacles[c0:c1], su.params,
                           name=su.name)
        parts.append(F.from_scene(sub, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, global_contact_solve=1,
                                  max_contacts=6000, use_graph=True))
        log(f"uneven full: created envs {c0}..{c1 - 1} ({sum(nv[c0:c1])} vertices) at "
            f"{time.perf_counter() - t0:.1f}s")
    create_s = time.perf_counter() - t0
    for b in parts:
        b.step(args.warmup)
    for b in parts:
        b.synchronize()
        b.residual_history(reset=True)
    t = time.perf_counter()
    for s_ in range(args.steps):
        for b in parts:
            b.step(1)
    for b in parts:
        b.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    mx, over, newton, st = 0.0, 0, 0, 0
    stats = []
    for b in parts:
        m_, o_, n_, s2 = b.residual_history(reset=True, full=True)
        mx, over, newton, st = max(mx, m_), over + o_, newton + n_, st + s2
        stats += b.stats()
    cts = np.array([s_["contacts"] for s_ in stats])
    res = np.array([s_["residual"] for s_ in stats])
    out = {"workload": f"uneven_batch: {ne} envs (seed 7), sheets 16^2-48^2 and tet blocks 500-8000 vertices, "
                       f"1-3 moving boxes or capsules each, K = 10, FP32, lightweight metric from global memory, "
                       f"budget 10 updates per local-global iteration, HIP graph, {len(parts)} stream groups of "
                       f"at most {chunk} envs",
           "vertices": int(sum(nv)), "largest_env_vertices": int(max(nv)), "create_s": round(create_s, 1),
           "ms_per_step": round(1e3 * dt, 3), "env_steps_per_s": round(ne / dt, 1),
           "updates_per_lg_iteration": round(newton / max(st, 1) / 10, 2),
           "contacts_per_env": {"mean": round(float(cts.mean()), 1), "max": int(cts.max())},
           "end_of_step_residual_m": {"median": float(f"{np.median(res):.3e}"), "p90": float(f"{np.quantile(res, 0.9):.3e}"),
                                      "max": float(f"{mx:.3e}")},
           "env_steps_above_ncp_tol": int(over), "env_steps": int(st)}
    # oracle check of the largest sheet and the largest block, one step from a history reset
    sheets = [e for e in range(ne) if su.envs[e].elem == scenes.TRI]
    blocks = [e for e in range(ne) if su.envs[e].elem == scenes.TET]
    pick = [max(sheets, key=lambda e: nv[e]), max(blocks, key=lambda e: nv[e])]
    xs, vs, obs, x1 = {}, {}, {}, {}
    for e in pick:
        b, le = parts[e // chunk], e % chunk
        x, v = b.get_state(env=le)
        b.set_state(x, v, env=le)
        xs[e], vs[e], obs[e] = x, v, b.get_obstacles(le)
    for b in parts:
        b.step(1)
    for e in pick:
        x1[e] = parts[e // chunk].get_state(env=e % chunk)[0]
    chk = {}
    for e in pick:
        oe = O.precompute(su.envs[e], su.params.h)
        # the FP32 batch's default inner tolerance: 0.25 ncp_tol
        ref = O.step_lightweight(oe, xs[e], vs[e], obs[e], su.params, newton_iterations=10,
                                 tol=0.25 * su.params.ncp_tol)
        L = np.linalg.norm(su.envs[e].rest_x.max(0) - su.envs[e].rest_x.min(0))
        err = float(np.abs(x1[e] - ref.x).max())
        chk[str(e)] = {"vertices": nv[e], "contacts": int(ref.contacts.count), "max_abs_m": float(f"{err:.3e}"),
                       "max_rel": float(f"{err / max(np.abs(ref.x).max(), L):.3e}")}
        log(f"uneven full: env {e} ({nv[e]} vertices, {ref.contacts.count} contacts) |dq| {err:.2e}")
    out["oracle_check_from_reset"] = chk
    for b in parts:
        b.close()
    return out


def squeeze_horizon(F, scenes, args):
    """The squeeze's whole horizon, from its first step, in the batched configuration."""
    n_steps, block = 500, 50
    sc = scenes.squeeze_blocks(args.envs, seed=0)
    t0 = time.perf_counter()
    b = F.from_scene(sc, warm_start=F.FLASH_WS_PREV, fused_lg=True)
    create_s = time.perf_counter() - t0
    b.synchronize()
    b.residual_history(reset=True)
    blocks = []
    t = time.perf_counter()
    for s0 in range(0, n_steps, block):
        t1 = time.perf_counter()
        b.step(block)
        b.synchronize()
        blocks.append(round(1e3 * (time.perf_counter() - t1) / block, 2))
        log(f"squeeze horizon: steps {s0}..{s0 + block - 1} {blocks[-1]} ms/step")
    dt = time.perf_counter() - t
    mx, failed, newton, env_steps = b.residual_history(reset=True, full=True)
    dropped = sum(1 for s_ in b.stats() if s_["flags"] & 4)
    b.close()
    assert dropped == 0, f"{dropped} envs dropped contacts beyond the capacity"
    return {"workload": f"squeeze_blocks: {args.envs} envs, steps 0..{n_steps - 1} (the whole horizon), the "
                        f"local-global loop as one launch per step, one stream, previous-step warm start, FP32 "
                        f"(contact-space solve FP64), every contact solve to NCP residual <= 1e-6",
            "env_steps_per_s": round(len(sc.envs) * n_steps / dt, 1), "ms_per_step": round(1e3 * dt / n_steps, 3),
            "ms_per_step_by_block_of_50": blocks, "max_residual": mx, "env_steps_failed": int(failed),
            "env_steps": int(env_steps), "newton_per_env_step": round(newton / max(env_steps, 1), 3),
            "create_s": round(create_s, 1)}


def slab_press(F, scenes, torch, args):
    """The large-scene recipe with shared inverses (64 copies of a 100k-vertex slab)."""
    from oracle import flash_oracle as O     # the oracle check of one env (test infrastructure)
    ne = args.slab_envs
    sc = scenes.slab_press(ne)
    os.environ["FLASH_PROGRESS"] = "1"        # the 100k-vertex inverse reports progress while it is formed
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    b = F.from_scene(sc, contact_metric=F.FLASH_METRIC_LIGHTWEIGHT, global_contact_solve=1, max_contacts=30000,
                     use_graph=True)
    create_s = time.perf_counter() - t0
    footprint = free0 - torch.cuda.mem_get_info()[0]
    log(f"slab press: created {ne} envs in {create_s:.1f}s, HBM footprint {footprint / 1e9:.1f} GB")
    for s_ in range(args.warmup):
        t = time.perf_counter()
        b.step(1)
        b.synchronize()
        log(f"slab press: warm-up step {s_} {time.perf_counter() - t:.2f}s")
    b.residual_history(reset=True)
    per = []
    for s_ in range(args.steps):
        t = time.perf_counter()
        b.step(1)
        b.synchronize()
        per.append(time.perf_counter() - t)
        log(f"slab press: timed step {s_} {per[-1]:.2f}s")
    dt = float(np.mean(per))
    mx, over, newton, st = b.residual_history(reset=True, full=True)
    stats = b.stats()
    cts = np.array([s_["contacts"] for s_ in stats])
    res = np.array([s_["residual"] for s_ in stats])
    n = sc.envs[0].n_vertices
    out = {"workload": f"slab_press: {ne} envs of a {n}-vertex, {sc.envs[0].n_elements}-tet slab (100 x 9 x 100 "
                       f"hexes of 5 mm) pressed 5 mm by two pads at 2 cm/s, FP32, lightweight metric from global "
                       f"memory, K = 10, budget 10, HIP graph, one shared explicit inverse",
           "create_s": round(create_s, 1), "hbm_footprint_gb": round(footprint / 1e9, 2),
           "ms_per_step": round(1e3 * dt, 3), "env_steps_per_s": round(ne / dt, 2),
           "timed_steps": [args.warmup, args.warmup + args.steps - 1],
           "updates_per_lg_iteration": round(newton / max(st, 1) / 10, 2),
           "contacts_per_env": {"mean": round(float(cts.mean()), 1), "max": int(cts.max())},
           "end_of_step_residual_m": {"median": float(f"{np.median(res):.3e}"), "max": float(f"{mx:.3e}")},
           "env_steps_above_ncp_tol": int(over), "env_steps": int(st),
           "inverse_bytes_per_product": 4 * n * ((n + 31) // 32 * 32)}
    x, v = b.get_state(env=0)
    b.set_state(x, v, env=0)
    obs = b.get_obstacles(0)
    b.step(1)
    x1 = b.get_state(env=0)[0]
    b.close()
    if args.slab_dump:
        # the oracle check of this state runs elsewhere (it takes minutes): env 0's state, its next
        # GPU step and the obstacles at that step
        np.savez(args.slab_dump, x=x, v=v, x1=x1, kind=np.array([o.kind for o in obs]),
                 center=np.array([o.center for o in obs]), rot=np.array([o.rot for o in obs]),
                 size=np.array([o.size for o in obs]), vel=np.array([o.lin_vel for o in obs]),
                 move=np.array([o.move_steps for o in obs]))
        out["oracle_check_from_reset"] = {"state_written_to": args.slab_dump}
        return out
    t1 = time.perf_counter()
    oe = O.precompute(sc.envs[0], sc.params.h)
    log(f"slab press: oracle precompute {time.perf_counter() - t1:.0f}s")
    ref = O.step_lightweight(oe, x, v, obs, sc.params, newton_iterations=10, tol=0.25 * sc.params.ncp_tol,
                             progress=lambda k: log(f"slab press: oracle local-global iteration {k} done"))
    L = np.linalg.norm(sc.envs[0].rest_x.max(0) - sc.envs[0].rest_x.min(0))
    err = float(np.abs(x1 - ref.x).max())
    out["oracle_check_from_reset"] = {"env": 0, "contacts": int(ref.contacts.count), "max_abs_m": float(f"{err:.3e}"),
                                      "max_rel": float(f"{err / max(np.abs(ref.x).max(), L):.3e}"),
                                      "oracle_s": round(time.perf_counter() - t1, 1)}
    log(f"slab press: env 0 against the oracle |dq| {err:.2e} ({ref.contacts.count} contacts)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--envs", type=int, default=1024)
    ap.add_argument("--arms", default=",".join(ALL_ARMS),
                    help="comma-separated subset of " + ",".join(ALL_ARMS) + " (opt-in: " + ",".join(OPT_IN_ARMS) + ")")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle steps per env in the CPU baseline")
    ap.add_argument("--cpu-procs", type=int, default=16, help="host processes of the all-cores CPU baseline")
    ap.add_argument("--groups", type=int, default=3, help="env groups on separate streams in batched_groups")
    ap.add_argument("--reset-every", type=int, default=5, help="steps between history drops in cold_starts")
    ap.add_argument("--uneven-envs", type=int, default=4096)
    ap.add_argument("--uneven-full-envs", type=int, default=1024)
    ap.add_argument("--slab-envs", type=int, default=64)
    ap.add_argument("--slab-dump", default="", help="write env 0's state for an offline oracle check instead")
    ap.add_argument("--fold-side", type=int, default=64, help="vertices per side of the folding sheet")
    ap.add_argument("--fold-warmup", type=int, default=20)
    ap.add_argument("--fold-steps", type=int, default=20)
    ap.add_argument("--fold-envs", type=lambda s: [int(v) for v in s.split(",")], default=list(FOLD_ENVS),
                    help="comma-separated env counts of the fold sweep")
    ap.add_argument("--profile-window", action="store_true",
                    help="pause the profiler except during the reported arm's timed steps (roctx)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 1 GiB device copy inside the profiled region (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: environments are independent and this build "
              "measures one GPU's share; see the design notes for how envs shard.", file=sys.stderr)
        sys.exit(2)
    arms_on = [a.strip() for a in args.arms.split(",") if a.strip()]
    for a in arms_on:
        if a not in ALL_ARMS + OPT_IN_ARMS:
            sys.exit(f"unknown arm {a}")
    # with --selected-regions the profiler starts paused: the first call is the window's resume
    roctx = Roctx(args.profile_window)

    import torch
    from paper_2604_17513_amd import flash as F
    from paper_2604_17513_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = 1 << 28
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        roctx.resume()
        c.copy_(a)
        torch.cuda.synchronize()
        roctx.pause()
        log(f"copy probe: {2 * 4 * n} bytes moved ({4 * n} read, {4 * n} written)")
        del a, c
    sc = scenes.squeeze_blocks(args.envs, seed=0)
    nv = [e.n_vertices for e in sc.envs]
    K = sc.params.lg_iterations
    sample = sorted({0, args.envs // 2, args.envs - 1})
    arms, checks = {}, {}
    head = None
    breakdown, apply_roof, schedule = None, None, None
    training, mlp_roof = None, None
    window_state = None

    if "plain" in arms_on:
        res, ex, jobs = run_arm(F, sc, args, warm_start=F.FLASH_WS_PREV, timing=0xFFFF, sample=sample,
                                check=not args.no_oracle_check,
                                capture=0 if args.no_cpu_baseline else min(args.cpu_procs, args.envs))
        window_state = ex["start_state"]
        kt = ex["kt"]
        apply_ms, apply_n = kt["apply"]
        apply_avg = apply_ms / max(apply_n, 1)
        bpl = apply_bytes_per_launch(nv)
        achieved = bpl / (apply_avg * 1e-3) / 1e9
        breakdown = {k: round(v[0] / args.steps, 3) for k, v in kt.items() if v[1]}
        schedule = ex["batch"].schedule_info()
        csrc = os.path.join(ROOT, "paper_2604_17513_amd", "csrc")
        gemv_hash = kernel_source_hash(os.path.join(csrc, "flash_kernels.hip"), "gemv_tile", "k_gemv")
        traffic = committed_traffic(os.path.join(ROOT, "profiles", "hbm_traffic_apply_squeeze_blocks_1024.md"),
                                    gemv_hash) if args.envs == 1024 else None
        apply_roof = {"bound": "hbm", "kernel": "batched global apply of the per-phase step (k_gemv<float,false>)",
                      "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "bytes_per_launch": bpl,
                      "bytes_note": "the full n x n inverse as stored (4 n^2 + 24 n per env)",
                      "avg_launch_ms": round(apply_avg, 4), "launches": apply_n, "kernel_source_sha256": gemv_hash}
        ex["batch"].close()
        arms["plain"] = res
        checks["plain"] = jobs
        log(f"plain arm: {res['ms_per_step']} ms/step")

    if "batched" in arms_on:
        res, ex, jobs = run_arm(F, sc, args, warm_start=F.FLASH_WS_PREV, fused=True, sample=sample,
                                check=not args.no_oracle_check)
        ex["batch"].close()
        arms["batched"] = res
        checks["batched"] = jobs
        log(f"batched arm: {res['ms_per_step']} ms/step")

    ws = None
    if any(a in arms_on for a in ("batched_learned", "batched_groups", "cold_starts")):
        w, nm, training = train_warm_start(F, scenes, torch)
        ws = (w, nm)
        log(f"trained warm start on {training['pairs']} pairs in {training['train_s']}s")

    if "batched_learned" in arms_on:
        res, ex, jobs = run_arm(F, sc, args, warm_start=F.FLASH_WS_LEARNED, ws=ws, fused=True, timing=K_FUSED_BIT,
                                roctx=roctx, sample=sample, check=not args.no_oracle_check)
        kt = ex["kt"]
        f_ms, f_n = kt["lg_fused"]
        contacts = [s_["contacts"] for s_ in ex["stats"]]
        nw = [ex["newton_per_env_step"]] * len(sc.envs)
        head = (res, ex, contacts, nw, f_ms / max(f_n, 1), f_n)
        ex["batch"].close()
        arms["batched_learned"] = res
        checks["batched_learned"] = jobs
        log(f"batched+learned arm: {res['ms_per_step']} ms/step")

    if "batched_groups" in arms_on:
        res, ex, jobs = run_arm(F, sc, args, warm_start=F.FLASH_WS_LEARNED, ws=ws, fused=True, use_graph=True,
                                groups=args.groups, sample=sample, check=not args.no_oracle_check)
        ex["batch"].close()
        res.update({"stream_groups": args.groups, "graphs": True})
        arms["batched_groups"] = res
        checks["batched_groups"] = jobs
        log(f"batched groups arm: {res['ms_per_step']} ms/step")

    if "cold_starts" in arms_on:
        cold = {"reset_every_steps": args.reset_every}
        for name, wsm in (("plain_start", F.FLASH_WS_PREV), ("learned_start", F.FLASH_WS_LEARNED)):
            res, ex, jobs = run_arm(F, sc, args, warm_start=wsm, ws=ws if wsm == F.FLASH_WS_LEARNED else None,
                                    fused=True, reset_every=args.reset_every, sample=sample,
                                    check=not args.no_oracle_check)
            ex["batch"].close()
            cold[name] = res
            checks["cold_starts." + name] = jobs
            log(f"cold starts, {name}: {res['ms_per_step']} ms/step, Newton {res['newton_per_env_step']}")
        cold["newton_gain"] = round(1.0 - cold["learned_start"]["newton_per_env_step"] /
                                    max(cold["plain_start"]["newton_per_env_step"], 1e-9), 4)
        cold["throughput_gain"] = round(cold["learned_start"]["env_steps_per_s"] /
                                        cold["plain_start"]["env_steps_per_s"] - 1.0, 4)
        arms["cold_starts"] = cold

    if ws is not None and "batched_learned" in arms_on:
        mlp_roof = mlp_roofline(F, torch)
        log(f"network forward: {mlp_roof['achieved']} TFLOP/s")

    if "uneven_batched" in arms_on and args.uneven_envs > 0:
        su = scenes.uneven_batch(args.uneven_envs, seed=7, max_tet_vertices=1200, max_cloth_side=17,
                                 lg_iterations=10)
        us = sorted({0, args.uneven_envs // 2, args.uneven_envs - 1})
        res, ex, jobs = run_arm(F, su, args, warm_start=F.FLASH_WS_PREV, fused=True, use_graph=True,
                                groups=args.groups, sample=us, check=not args.no_oracle_check)
        ex["batch"].close()
        res.update({"workload": f"uneven_batch: {args.uneven_envs} envs (seed 7), cloth sheets 16^2-17^2 and tet "
                                f"blocks of 500-1200 vertices, 1-3 moving boxes or capsules each, K=10, FP32",
                    "vertices": int(sum(e.n_vertices for e in su.envs)), "stream_groups": args.groups})
        arms["uneven_batched"] = res
        checks["uneven_batched"] = jobs
        log(f"uneven batched arm: {res['ms_per_step']} ms/step")

    if "fold_sweep" in arms_on:
        arms["fold_sweep"] = fold_sweep(F, scenes, args)

    if "depth_render" in arms_on:
        arms["depth_render"] = depth_render(F, scenes, torch, args)

    if "uneven_full" in arms_on:
        arms["uneven_full"] = uneven_full(F, scenes, args)

    if "slab_press" in arms_on:
        arms["slab_press"] = slab_press(F, scenes, torch, args)

    if "squeeze_horizon" in arms_on:
        arms["squeeze_horizon"] = squeeze_horizon(F, scenes, args)

    if "contact_metric" in arms_on:
        arms["contact_metric"] = metric_compare(F, scenes, args)
        c2 = [v for k, v in arms["contact_metric"].items() if k.startswith("C2")][0]
        log("contact metric: " + ", ".join(f"{k} {v['updates_per_lg_iteration']} updates, {v['ms_per_step']} ms"
                                           for k, v in c2.items()))

    cpu = None
    # ---- host legs (spawned processes: the GPU state of this process is not inherited)
    model, ncpu, avail = cpu_info()
    oracle_error = {}
    flat = [(arm, j) for arm, js in checks.items() for j in js]
    if flat:
        with spawn_pool(min(len(flat), max(1, min(avail, 16)))) as pool:
            outs = pool.starmap(_oracle_check, [j for _, j in flat])
        for (arm, _), (err, rel, same, r) in zip(flat, outs):
            o = oracle_error.setdefault(arm, {"envs_checked": 0, "max_abs_m": 0.0, "max_rel": 0.0,
                                              "oracle_residual_of_gpu_step": 0.0, "same_contacts": True})
            o["envs_checked"] += 1
            o["max_abs_m"] = max(o["max_abs_m"], err)
            o["max_rel"] = max(o["max_rel"], rel)
            o["oracle_residual_of_gpu_step"] = max(o["oracle_residual_of_gpu_step"], r)
            o["same_contacts"] = o["same_contacts"] and same
        for arm, o in oracle_error.items():
            tgt = arms[arm.split(".")[0]]
            if "." in arm:
                tgt = tgt[arm.split(".")[1]]
            tgt["oracle_error"] = {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in o.items()}
    if window_state is not None:
        xs0, vs0, obs = window_state
        procs = max(1, min(args.cpu_procs, avail, args.envs))
        n_steps = args.cpu_steps
        job = lambda e, thr: (sc.envs[e], xs0[e], vs0[e], obs[e], sc.params, n_steps, thr)  # noqa: E731
        t0 = time.time()
        with spawn_pool(1) as pool:
            pool.map(_warm_imports, [0])
            (t_one, _), = pool.starmap(_oracle_job, [job(0, 1)])
        with spawn_pool(procs) as pool:
            pool.map(_warm_imports, range(procs))
            t_all = time.time()
            pool.starmap(_oracle_job, [job(e, 1) for e in range(procs)])
            t_all = time.time() - t_all
        cpu = {
            "value": round(procs * n_steps / t_all, 3),
            "unit": "env-steps/s",
            "cores": procs,
            "kind": "oracle",
            "value_1_thread": round(n_steps / t_one, 3),
            "cpu_model": model,
            "nproc": ncpu,
            "cpus_available": avail,
            "sample": f"envs 0..{procs - 1} of the timed workload from the GPU's state at step {args.warmup} (the "
                      f"start of the timed window), {n_steps} oracle steps each; all cores: {procs} processes with "
                      f"one BLAS thread each ({t_all:.1f}s wall); 1 thread: env 0 alone ({t_one:.1f}s); "
                      f"exact-Delassus FP64 oracle, unoptimised",
        }
        log(f"cpu baseline: {cpu['value']} env-steps/s on {procs} processes, {cpu['value_1_thread']} on 1 thread "
            f"({time.time() - t0:.0f}s)")

    # ---- the reported line
    if head is not None:
        res, ex, contacts, nw, f_avg, f_n = head
        value_arm = "batched_learned"
    else:
        # only the arms timed on the squeeze's window describe this line's workload
        window_arms = ("plain", "batched", "batched_groups", "cold_starts")
        first = next((a for a in window_arms if a in arms), None)
        if first is None:
            print(json.dumps({"metric": METRIC, "value": None, "unit": "env-steps/s", "n_gpus": 1,
                              "note": "no arm of the headline workload ran", "arms": arms}))
            return
        res, value_arm = arms[first], first
    value = res["env_steps_per_s"] if value_arm != "cold_starts" else res["learned_start"]["env_steps_per_s"]
    ms_per_step = res["ms_per_step"] if value_arm != "cold_starts" else res["learned_start"]["ms_per_step"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"squeeze_blocks: {args.envs} envs x 10^3-hex block (1331 v, 6000 tets), two box fingers + "
                        f"ground, h=1/60, K=20 local-global iterations, FP32 (contact-space solve FP64), every contact "
                        f"solve to NCP residual <= 1e-6; timed steps {args.warmup}-{args.warmup + args.steps - 1} of "
                        f"the squeeze",
            "arm_reported_as_value": value_arm,
            "n_envs": args.envs,
            "vertices_per_env": nv[0],
            "tets_per_env": int(sc.envs[0].n_elements),
            "lg_iterations": K,
            "ncp_tol": sc.params.ncp_tol,
        },
    }
    if head is not None:
        res, ex, contacts, nw, f_avg, f_n = head
        out["config"]["contacts_per_env_mean"] = round(float(np.mean(contacts)), 1)
        per_step = path_bytes(sc.envs, contacts, K, nw)
        over_step = overhead_bytes(sc.envs, contacts, K)
        achieved = per_step / (f_avg * 1e-3) / 1e9
        csrc = os.path.join(ROOT, "paper_2604_17513_amd", "csrc")
        fused_hash = source_hash(os.path.join(csrc, "flash_kernels.hip"), os.path.join(csrc, "flash_device.h"),
                                 os.path.join(csrc, "flash_contact.h"))
        traffic = committed_traffic(os.path.join(ROOT, "profiles", "hbm_traffic_lg_fused_squeeze_blocks_1024.md"),
                                    fused_hash) if args.envs == 1024 else None
        out["roofline"] = {
            "bound": "hbm",
            "kernel": "k_lg_fused<float,double>: K x (projection, assembly, global apply, contact solve, position "
                      "update), one workgroup per env, one launch per step, in the reported arm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": per_step,
            "overhead_bytes_per_launch": over_step,
            "bytes_formula": "sum over envs of 24 n_v + 64 n_c + K (56 n_tet + 36 n_v + 8 n_v (n_v + 1) / 2 + 36 n_v) "
                             "+ N_newton 108 n_c + 48 n_v",
            "newton_per_env_step": round(nw[0], 3),
            "avg_launch_ms": round(f_avg, 4),
            "launches": f_n,
            "timed_steps": [args.warmup, args.warmup + args.steps - 1],
            "kernel_source_sha256": fused_hash,
        }
    if apply_roof is not None:
        out["roofline_apply"] = apply_roof
    # arms that solve every contact problem to the NCP tolerance (the fixed-budget and rendering arms
    # report their own residuals)
    tol_arms = [a for k, a in arms.items() if k in ("plain", "batched", "batched_learned", "batched_groups",
                                                    "cold_starts", "uneven_batched")]
    mx = max([a["max_residual"] if "max_residual" in a else max(a["plain_start"]["max_residual"],
                                                                 a["learned_start"]["max_residual"])
              for a in tol_arms] or [0.0])
    failed = sum(a["env_steps_failed"] if "env_steps_failed" in a else
                 a["plain_start"]["env_steps_failed"] + a["learned_start"]["env_steps_failed"] for a in tol_arms)
    out["max_residual"] = mx
    out["env_steps_failed"] = failed
    out["residual_ok"] = bool(mx <= sc.params.ncp_tol and failed == 0)
    out["arms"] = arms
    if breakdown is not None:
        out["kernel_ms_per_step_plain"] = breakdown
    if schedule is not None:
        out["apply_schedule"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in schedule.items()
                                 if k != "candidate_ms"}
    if mlp_roof is not None:
        out["roofline_network"] = mlp_roof
    if training is not None:
        out["warm_start_training"] = training
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()

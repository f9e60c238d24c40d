"""Throughput of the MUFFIN iteration on one MI355X: voxel-iterations per second.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube1024_L256_J5] [--no-cpu]

One step is one full iteration of Algorithm 1 over the whole cube (spatial adjoint, gradient,
fused spectral step, spatial dual step).  Inputs are synthetic (seeded generator), uploaded to HBM
before timing.  Prints one JSON line.  Other workloads: --workload batch32 (32 uneven cubes
advanced together), --workload cnn (the warm-start network's inference and training step),
--workload calib (the mu_lambda = 0 first step of the calibration protocol of Sec. 4, beside the
learned warm start's inference time on the same cube), --workload vis (the iteration with the
visibility-domain data term of Sec. 2, eq. (viseq), on 256^2 x 64 channels and 2000 baselines).
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def alg_bytes_per_voxel(N, J, spectral=True):
    """Compulsory HBM bytes per voxel-iteration of the two-phase iteration (FP32 state):
    U read+write 8(J+1), X 12 (read in the gradient, read and written in the primal step), V read+write
    8, b 4, |H|^2 2(N+2)/N (half spectrum, FP32), q write+read 8, d write+read 8: 40 + 8(J+1) + 2(N+2)/N.
    Without the spectral step (mu_lambda = 0) V and the q exchange drop out: 24 + 8(J+1) + 2(N+2)/N."""
    return (40.0 if spectral else 24.0) + 8.0 * (J + 1) + 2.0 * (N + 2) / N


# Algorithmic bytes per voxel that each hot kernel moves, counting only the terms of the iteration's
# bytes model above, each charged to the launch that moves it first (re-reads of U and intermediate
# planes count nothing), at J = 5 with the fused tail: the gradient's passes x 4, |H|^2 2(N+2)/N,
# b + q 8; the spectral step X 8, V 8, q 4, d 4; the analysis triple d 4 and u_0..u_2 24; the fused
# tail u_3, u_4 and the coarse plane 24; the adjoint triple 0.  They sum to the bytes model.
def kernel_alg_bytes(name, N):
    table = {
        "k_spectral_fft (fused spectral step)": 24.0,
        "k_triple_an<RS, false> (three scales of analysis + spatial dual steps)": 28.0,
        "k_fused<RS> (last analysis pair + next iteration's first adjoint pair)": 24.0,
        "k_triple_adj<RS> (three adjoint Horner steps)": 0.0,
        "k_rows_r2c": 4.0,
        "k_cols<REAL>": 2.0 * (N + 2) / N,
        "k_rows_c2r<GRAD>": 8.0,
    }
    return table.get(name)


# Bytes per voxel of one launch of each hot kernel as scheduled (what it reads and writes, including
# re-reads and intermediate planes), and its slot k in the library's profile (mean launch time at
# 8 + 2k, launches per iteration at 9 + 2k)
KERNEL_BYTES = {
    # reads x, q, V and writes x, d, V
    "k_spectral_fft (fused spectral step)": 24.0,
    # reads c_j and u_j, writes c_{j+1} and u_j
    "k_band<DB_ANALYSIS> (one scale of analysis + spatial dual step)": 16.0,
    # reads u_j and the running adjoint sum a, writes the new sum
    "k_band<DB_ADJOINT> (one scale of the adjoint Horner step)": 12.0,
    # reads c_{J-1}, u_{J-1} and the coarse dual u_J, writes u_{J-1} and u_J
    "k_band<DB_ANALYSIS_C> (last scale of analysis + spatial and coarse dual steps)": 20.0,
    # reads c_j, u_j, u_{j+1}, writes u_j, u_{j+1}, c_{j+2}
    "k_pair<PR_ANALYSIS> (two scales of analysis + spatial dual steps)": 24.0,
    # reads u_{j+1}, u_j and a, writes the new sum
    "k_pair<PR_ADJOINT> (two adjoint Horner steps)": 16.0,
    # reads c_{J-2}, u_{J-2}, u_{J-1}, u_J, writes u_{J-2}, u_{J-1}, u_J
    "k_pair<PR_ANALYSIS_C> (last two analysis scales + spatial and coarse dual steps)": 28.0,
    # reads c_j, u_j, u_{j+1}, u_{j+2}, writes u_j, u_{j+1}, u_{j+2}, c_{j+3}
    "k_triple_an<RS, false> (three scales of analysis + spatial dual steps)": 32.0,
    # reads u_{j+2}, u_{j+1}, u_j and a, writes the new sum
    "k_triple_adj<RS> (three adjoint Horner steps)": 20.0,
    # reads c_{J-3}, the three u planes and u_J, writes the three u planes and u_J
    "k_triple_an<RS, true> (last three analysis scales + spatial and coarse dual steps)": 36.0,
    # reads c_{J-2} and the old u_{J-2}, u_{J-1}, u_J; writes the new ones and the adjoint sum after
    # the next iteration's first two Horner steps
    "k_fused<RS> (last analysis pair + next iteration's first adjoint pair)": 32.0,
}
PROFILE_SLOT = {
    "k_band<DB_ANALYSIS> (one scale of analysis + spatial dual step)": 0,
    "k_band<DB_ADJOINT> (one scale of the adjoint Horner step)": 1,
    "k_band<DB_ANALYSIS_C> (last scale of analysis + spatial and coarse dual steps)": 2,
    "k_pair<PR_ANALYSIS> (two scales of analysis + spatial dual steps)": 3,
    "k_pair<PR_ADJOINT> (two adjoint Horner steps)": 4,
    "k_pair<PR_ANALYSIS_C> (last two analysis scales + spatial and coarse dual steps)": 5,
    "k_triple_an<RS, false> (three scales of analysis + spatial dual steps)": 6,
    "k_triple_adj<RS> (three adjoint Horner steps)": 7,
    "k_triple_an<RS, true> (last three analysis scales + spatial and coarse dual steps)": 8,
    "k_fused<RS> (last analysis pair + next iteration's first adjoint pair)": 9,
}


# HBM bytes per launch of the hot kernels, from two rocprofv3 --pmc runs of this script (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) on the named workload: the mean over the kernel's launches,
# times the factor a 1 GiB elementwise copy (--calib-copy) gives for the same counter.  An entry
# holds only for the source files that define the kernel as they were when it was taken (hash
# below); otherwise traffic is null.
MEASURED_TRAFFIC = {
    "k_fused<RS> (last analysis pair + next iteration's first adjoint pair)": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/iuwt.hip"
        ],
        "sha256": "689ff4a1d518f22a",
        "fetch_kib": 2900091.0,
        "write_kib": 4194304.0,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_triple_an<RS, false> (three scales of analysis + spatial dual steps)": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/iuwt.hip"
        ],
        "sha256": "689ff4a1d518f22a",
        "fetch_kib": 2201709.1,
        "write_kib": 4194304.0,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_triple_adj<RS> (three adjoint Horner steps)": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/iuwt.hip"
        ],
        "sha256": "689ff4a1d518f22a",
        "fetch_kib": 2191451.5,
        "write_kib": 1048576.0,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_spectral_fft (fused spectral step)": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/spectral.hip",
            "paper_1602_08847_amd/csrc/fft_core.h"
        ],
        "sha256": "7dd811dd6ba2ef20",
        "fetch_kib": 1573104.7,
        "write_kib": 3145812.9,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_rows_r2c": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/fft.hip",
            "paper_1602_08847_amd/csrc/fft_core.h"
        ],
        "sha256": "7deb0bda57c04e0f",
        "fetch_kib": 524379.9,
        "write_kib": 1056768.3,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_cols<REAL>": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/fft.hip",
            "paper_1602_08847_amd/csrc/fft_core.h"
        ],
        "sha256": "7deb0bda57c04e0f",
        "fetch_kib": 831820.8,
        "write_kib": 1131519.9,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    },
    "k_rows_c2r<GRAD>": {
        "workload": "cube1024_L256_J5",
        "sources": [
            "paper_1602_08847_amd/csrc/fft.hip",
            "paper_1602_08847_amd/csrc/fft_core.h"
        ],
        "sha256": "7deb0bda57c04e0f",
        "fetch_kib": 1588558.7,
        "write_kib": 1048576.0,
        "fetch_factor": 1.9999,
        "write_factor": 1.0
    }
}


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """Counter-derived HBM bytes per launch of kernel, or None if not taken on these sources."""
    m = MEASURED_TRAFFIC.get(kernel)
    if not m or m["workload"] != workload or sources_sha256(m["sources"]) != m["sha256"]:
        return None
    return m["fetch_kib"] * 1024 * m["fetch_factor"] + m["write_kib"] * 1024 * m["write_factor"]


def cpu_baseline(spec, L_sample, iters, out_npz):
    """Time the FP64 oracle on a channel sample of the workload (same generator and image side, the
    first L_sample channels of a cube of that many channels) in a single-threaded subprocess, from a
    seeded positive X0 so that the positive part clips; its final state and step size go to out_npz
    for the parity check of the same sample on the GPU."""
    code = f"""
import time, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle import muffin as om
from paper_1602_08847_amd import synth
spec = synth.CubeSpec(N={spec.N}, L={L_sample}, J={spec.J}, n_sources={spec.n_sources},
                      n_baselines={spec.n_baselines}, seed={spec.seed})
c = synth.make_cube(spec, dtype=np.float32, with_sky=False)
rng = np.random.default_rng(7)
X0 = np.abs(rng.standard_normal(size=c.dirty.shape, dtype=np.float32)) * np.float32(8.0 * c.dirty.std())
p = om.Problem(dirty=c.dirty.astype(np.float64), psf=c.psf.astype(np.float64), J={spec.J}, mu_s=0.25, mu_l=3.0)
tau = om.step_sizes(p)[0]
st = om.init_state(p, X0.astype(np.float64))
t0 = time.perf_counter()
for _ in range({iters}):
    st = om.iterate(p, st, tau)
dt = time.perf_counter() - t0
np.savez({out_npz!r}, X=st.X, U=st.U, V=st.V, X0=X0, tau=tau, f=om.objective(p, st.X))
print(dt)
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    dt = float(out.stdout.strip().splitlines()[-1])
    return spec.N * spec.N * L_sample * iters / dt, dt


def sample_parity(muffin, spec, L_sample, iters, npz, flags):
    """The same channel sample on the GPU, in the timed launch configuration (the autotuned band rows
    of this process, the fused tail forced on), from the oracle's X0 with its tau: relative L2 errors
    of X, U, V and the relative objective error after the same iterations."""
    from paper_1602_08847_amd import synth
    ref = np.load(npz)
    c = synth.make_cube(synth.CubeSpec(N=spec.N, L=L_sample, J=spec.J, n_sources=spec.n_sources,
                                       n_baselines=spec.n_baselines, seed=spec.seed), dtype=np.float32, with_sky=False)
    with muffin.Muffin(c.dirty, c.psf, J=spec.J, mu_s=0.25, mu_lambda=3.0, tau=float(ref["tau"]), flags=flags) as m:
        m.set_x(ref["X0"])
        m.step(iters)
        got = {"X": m.get_x(), "U": m.get_u(), "V": m.get_v()}
        f = m.objective()[0]
    err = {}
    for k, t in got.items():
        a = t.double().cpu().numpy()
        err[k] = float(np.linalg.norm(a - ref[k]) / np.linalg.norm(ref[k]))
    err["objective"] = float(abs(f - ref["f"][0]) / abs(ref["f"][0]))
    err["clipped_fraction_X"] = float(np.mean(ref["X"] == 0))
    return err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cube1024_L256_J5")
    ap.add_argument("--gen", type=int, default=2)
    ap.add_argument("--flags", type=int, default=0, help="library flags (1: one IUWT scale per launch, 2: no fused tail, 4: fused tail)")
    ap.add_argument("--prior", choices=["iuwt", "uob"], default="iuwt",
                    help="spatial prior: the IUWT, or the union of the first 8 Daubechies bases")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=6)
    ap.add_argument("--autotune", type=int, default=1, help="1: tune the band kernels' row bands first")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB elementwise copy first (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1602_08847_amd import muffin, synth

    if args.workload.startswith("batch"):
        return bench_batch(args)
    if args.workload == "cnn":
        return bench_cnn(args)
    if args.workload == "calib":
        return bench_calib(args)
    if args.workload.startswith("vis"):
        return bench_vis(args)
    spec = synth.WORKLOADS[args.workload]
    N, L, J = spec.N, spec.L, spec.J
    t0 = time.time()
    cube = synth.make_cube(spec, dtype=np.float32, with_sky=False)
    gen_s = time.time() - t0
    print(f"[bench] generated {args.workload} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    dirty = torch.from_numpy(cube.dirty).cuda()
    psf = torch.from_numpy(cube.psf).cuda()
    del cube
    prior = muffin.PRIOR_UOB if args.prior == "uob" else muffin.PRIOR_IUWT
    m = muffin.Muffin(dirty, psf, J=J, mu_s=0.25, mu_lambda=3.0, iuwt_gen=args.gen, flags=args.flags, prior=prior)
    if prior == muffin.PRIOR_UOB:
        return bench_uob(args, m, spec)
    del dirty, psf
    torch.cuda.synchronize()
    print(f"[bench] context ready, tau={m.info()['tau']:.3e}", file=sys.stderr, flush=True)
    tune = m.autotune(reps=3) if args.autotune else None
    if tune:
        tiles = [(s['j'], s['kernel'], s['rows'], s['class_groups']) for s in json.loads(tune)['scales']]
        print(f"[bench] autotuned (scale, kernel, band rows, class groups): {tiles}", file=sys.stderr, flush=True)
    # the parity sample runs the timed kernels: the fused tail as the timed context has it
    fused = json.loads(tune).get("fused_tail") if tune else None
    sample_flags = args.flags if fused is None else (args.flags & ~6) | (4 if fused else 2)

    if args.calib_copy:
        # an elementwise kernel (not a DMA copy) that reads 1 GiB and writes 1 GiB
        src_t = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        torch.neg(src_t, out=dst_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    # per-phase and per-launch device times (eager launches, HIP events on the library stream)
    ph = m.profile(args.profile_steps)
    m.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = m.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = dev_ms / args.steps
    value = N * N * L * args.steps / (dev_ms / 1e3)
    obj = m.objective()
    print(f"[bench] {args.steps} steps: device {dev_ms:.2f} ms, wall {wall * 1e3:.2f} ms, "
          f"objective {obj[0]:.6e}; phases ms {np.round(ph[:5], 3).tolist()}", file=sys.stderr, flush=True)

    vox = N * N * L
    fams = {"k_spectral_fft (fused spectral step)": (ph[3], 1.0)}
    for name, k in PROFILE_SLOT.items():
        if ph[9 + 2 * k] > 0:
            fams[name] = (ph[8 + 2 * k], ph[9 + 2 * k])
    dom = max(fams, key=lambda k: fams[k][0] * fams[k][1])
    k_ms = fams[dom][0]
    b_k = kernel_alg_bytes(dom, N)
    sched_k = KERNEL_BYTES[dom]
    b_alg = alg_bytes_per_voxel(N, J)
    traffic = measured_traffic(dom, args.workload)
    if b_k is None:
        # the per-kernel split of the bytes model is written for the J = 5 schedule with the fused
        # tail; other schedules report the iteration as a whole
        dom_label, b_k, k_ms_used, traffic = "iteration (all launches)", b_alg, ms_per_step, None
    else:
        dom_label, k_ms_used = dom, k_ms
    k_gbs = b_k * vox / (k_ms_used * 1e-3) / 1e9
    roof = {
        "bound": "hbm",
        "kernel": dom_label,
        "achieved": round(k_gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(k_gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (fetch + write, rocprofv3 counters, calibrated)",
        "kernel_alg_bytes_per_voxel": b_k,
        "kernel_alg_bytes_per_launch": b_k * vox,
        "kernel_avg_ms": round(k_ms_used, 4),
        "longest_launch_family": dom,
        "kernel_schedule_bytes_per_voxel": sched_k,
        "kernel_schedule_gbs": round(sched_k * vox / (k_ms * 1e-3) / 1e9, 1),
        "iteration_alg_bytes_per_voxel": round(b_alg, 3),
        "iteration_alg_frac": round(b_alg * vox / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {"adjoint": round(ph[1], 3), "gradient": round(ph[2], 3),
                     "spectral": round(ph[3], 3), "analysis_dual": round(ph[4], 3)},
        "launch_ms": {name: [round(v[0], 4), v[1]] for name, v in fams.items()},
    }
    m.close()
    cpu = None
    if not args.no_cpu:
        import tempfile
        L_s, its = min(L, 12), 2
        with tempfile.TemporaryDirectory() as td:
            npz = os.path.join(td, "oracle_sample.npz")
            v, dt = cpu_baseline(spec, L_s, its, npz)
            err = sample_parity(muffin, spec, L_s, its, npz, flags=sample_flags)
        print(f"[bench] oracle sample {dt:.1f}s; FP32 vs FP64 errors {err}", file=sys.stderr, flush=True)
        cpu = {"value": v, "unit": "voxel-iter/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle, {N}x{N}x{L_s} channels of the same generator, J={J}, "
                         f"{its} iterations from a seeded positive X0, {dt:.1f}s single-threaded",
               "fp64_error": {**err, "what": f"relative L2 of the GPU's FP32 X, U, V after the same {its} "
                                             f"iterations of the same sample, autotuned band rows and fused "
                                             f"tail as timed, and the relative objective error"}}
    line = {
        "metric": f"voxel-iterations/s on {N}^2x{L} cube (MUFFIN primal-dual iteration)",
        "value": value,
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "L": L, "J": J, "iuwt_gen": args.gen,
                   "sources": spec.n_sources, "baselines": spec.n_baselines, "flags": args.flags},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_uob(args, m, spec):
    """The iteration with the union-of-bases prior (8 Daubechies bases, J levels) on the same cube:
    iteration throughput and per-phase device times; its bytes model replaces the IUWT's J + 1 dual
    planes by 8."""
    import torch
    N, L, J = spec.N, spec.L, spec.J
    ph = m.profile(args.profile_steps)
    m.step(args.warmup)
    torch.cuda.synchronize()
    dev_ms = m.step_timed(args.steps)
    torch.cuda.synchronize()
    ms_per_step = dev_ms / args.steps
    vox = N * N * L
    b_alg = 40.0 + 8.0 * 8 + 2.0 * (N + 2) / N
    m.close()
    line = {
        "metric": f"voxel-iterations/s on {N}^2x{L} cube, union-of-bases prior (8 Daubechies bases)",
        "value": vox * args.steps / (dev_ms / 1e3),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "L": L, "J": J, "prior": "uob"},
        "iteration_alg_bytes_per_voxel": round(b_alg, 3),
        "iteration_alg_frac": round(b_alg * vox / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {"adjoint": round(ph[1], 3), "gradient": round(ph[2], 3), "spectral": round(ph[3], 3),
                     "analysis_dual": round(ph[4], 3)},
    }
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """32 independent cubes of uneven sizes advanced together (one graph per image side)."""
    import torch
    from paper_1602_08847_amd import muffin, synth

    specs = synth.uneven_batch_specs(32, J=4)
    t0 = time.time()
    cubes = [synth.make_cube(s, dtype=np.float32, with_sky=False) for s in specs]
    print(f"[bench] generated 32 uneven cubes in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    vox = sum(s.N * s.N * s.L for s in specs)
    b = muffin.Batch([(c.dirty, c.psf) for c in cubes], J=4, mu_s=0.25, mu_lambda=3.0, flags=args.flags)
    del cubes
    tune = b.autotune(reps=3) if args.autotune else None
    b.step(args.warmup)
    torch.cuda.synchronize()
    dev_ms = b.step_timed(args.steps)
    ms_per_step = dev_ms / args.steps
    line = {
        "metric": "voxel-iterations/s, 32 uneven cubes in one batch (MUFFIN primal-dual iteration)",
        "value": vox * args.steps / (dev_ms / 1e3),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch32_uneven_J4", "cubes": [[s.N, s.L] for s in specs], "voxels": vox, "J": 4,
                   "autotuned": bool(args.autotune)},
        "iteration_alg_frac": round(sum(alg_bytes_per_voxel(s.N, 4) * s.N * s.N * s.L for s in specs)
                                    / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    print(json.dumps(line), flush=True)
    b.close()


def bench_calib(args):
    """The first step of the paper's calibration protocol (Sec. 4) on the 1024^2 x 256, J = 5 cube:
    mu_lambda = 0, so every channel iterates on its own (the primal step runs in the gradient's last
    pass and the spectral step is skipped), timed like the main workload; beside it, the time of the
    learned warm start (network inference) on the same cube, the other way to produce a starting
    point for the full method."""
    import torch
    from paper_1602_08847_amd import muffin, synth

    spec = synth.WORKLOADS["cube1024_L256_J5"]
    N, L, J = spec.N, spec.L, spec.J
    cube = synth.make_cube(spec, dtype=np.float32, with_sky=False)
    m = muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=0.25, mu_lambda=0.0, flags=args.flags)
    net = muffin.Cnn(seed=1)
    m2 = muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=0.25, mu_lambda=3.0)
    del cube
    if args.autotune:
        m.autotune(reps=3)
    ph = m.profile(args.profile_steps)
    m.step(args.warmup)
    torch.cuda.synchronize()
    dev_ms = m.step_timed(args.steps)
    torch.cuda.synchronize()
    ms_per_step = dev_ms / args.steps
    vox = N * N * L
    b_alg = alg_bytes_per_voxel(N, J, spectral=False)
    m.close()
    for _ in range(2):
        m2.warm_start(net)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        m2.warm_start(net)
    torch.cuda.synchronize()
    ws_ms = (time.perf_counter() - t0) * 1e3 / reps
    m2.close()
    net.close()
    line = {
        "metric": "voxel-iterations/s of the mu_lambda = 0 calibration step on the 1024^2x256 cube",
        "value": vox * args.steps / (dev_ms / 1e3),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "calib_step1_cube1024_L256_J5", "N": N, "L": L, "J": J, "mu_lambda": 0.0},
        "iteration_alg_bytes_per_voxel": round(b_alg, 3),
        "iteration_alg_frac": round(b_alg * vox / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {"adjoint": round(ph[1], 3), "gradient_and_primal_step": round(ph[2], 3),
                     "analysis_dual": round(ph[4], 3)},
        "step1_2000_iterations_s": round(2000 * ms_per_step / 1e3, 2),
        "cnn_warm_start_ms": round(ws_ms, 2),
    }
    print(json.dumps(line), flush=True)


# Visibility workload: the medium cube's shape (256^2 x 64 channels, J = 4, 2000 baselines) with the
# data term of eq. (viseq).  Each (visibility, pixel) pair needs at least two FP64 FMAs for the phase,
# one v_fract_f64, one conversion to FP32, one v_sin_f32, one v_cos_f32 and two FP32 FMAs: eight VALU
# instructions.  A SIMD issues one wave64 VALU instruction per four cycles (16 lanes a cycle), the
# sine and cosine included: their longer latency overlaps independent work (an issue-rate probe of
# this mix reached 9.3 lane slots per pair with its extra conversion).  256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = 3.93e13 lane slots per second, so 4.92e12 pairs per second bounds the direct sum.
VIS_SPEC = dict(N=256, L=64, K=2000, J=4, n_sources=20, seed=0)
VIS_SLOTS_PER_PAIR = 8.0
VIS_PAIR_PEAK = 256 * 4 * 16 * 2.4e9 / VIS_SLOTS_PER_PAIR
VIS_SAMPLE_TAU = 1e-6  # step of the FP64 sample (fixed, so that the oracle computes no beta)


def vis_regularisation(K):
    # the image-plane workloads' weights (mu_s 0.25, mu_lambda 3 for PSFs of peak 1) scaled by the
    # peak K of Phi^H Phi's point response; sigma keeps sigma ||K||^2 of the order of beta / 2
    return dict(mu_s=0.25 * K, mu_lambda=3.0 * K, sigma=1.0 / (4.0 * K))


def cpu_baseline_vis(L_sample, out_npz):
    """The FP64 oracle on the first L_sample channels of the visibility workload (single-threaded
    subprocess): visibilities simulated by the oracle's Phi plus the generator's noise, then one
    iteration from a seeded positive X0 with a fixed tau; its inputs and final state go to out_npz
    for the same sample on the GPU."""
    sp = VIS_SPEC
    code = f"""
import time, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle import muffin as om, visibility as ov
from paper_1602_08847_amd import synth
vi = synth.make_vis_inputs(synth.VisSpec(N={sp['N']}, L={sp['L']}, K={sp['K']}, n_sources={sp['n_sources']},
                                         seed={sp['seed']}))
Ls = {L_sample}
lam = vi.lam[:Ls]
vis = np.stack([ov.phi(vi.sky[l:l + 1], vi.uvw, lam[l:l + 1], vi.cell)[0] for l in range(Ls)]) + vi.noise[:Ls]
vis = vis.astype(np.complex64).astype(np.complex128)
d = ov.VisData(uvw=vi.uvw, lam=lam, cell=vi.cell, vis=vis, N={sp['N']})
reg = {vis_regularisation(sp['K'])!r}
p = om.Problem(dirty=None, psf=None, J={sp['J']}, mu_s=reg['mu_s'], mu_l=reg['mu_lambda'], sigma=reg['sigma'], vis=d)
rng = np.random.default_rng(7)
X0 = np.abs(rng.standard_normal(size=(Ls, {sp['N']}, {sp['N']}), dtype=np.float32))
st = om.init_state(p, X0.astype(np.float64))
t0 = time.perf_counter()
st = om.iterate(p, st, {VIS_SAMPLE_TAU!r})
dt = time.perf_counter() - t0
np.savez({out_npz!r}, X=st.X, U=st.U, V=st.V, X0=X0, vis=vis, lam=lam)
print(dt)
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    dt = float(out.stdout.strip().splitlines()[-1])
    return sp["N"] * sp["N"] * L_sample / dt, dt


def bench_vis(args):
    """The iteration of Algorithm 1 with the visibility-domain data term (Sec. 2, eq. (viseq)):
    exact Phi and Phi^H by direct sums on the GPU.  The timed workload's visibilities are the
    library's own Phi of the synthetic sky plus the generator's noise (their values do not change
    the work); the FP64 sample's come from the oracle."""
    import torch
    from paper_1602_08847_amd import muffin, synth
    sp = VIS_SPEC
    N, L, K, J = sp["N"], sp["L"], sp["K"], sp["J"]
    vi = synth.make_vis_inputs(synth.VisSpec(N=N, L=L, K=K, n_sources=sp["n_sources"], seed=sp["seed"]))
    reg = vis_regularisation(K)
    with muffin.Muffin.from_visibilities(np.zeros((L, K), np.complex64), vi.uvw, vi.lam, vi.cell, N=N, J=J,
                                         power_iters=1, **reg) as m0:
        v = m0.apply_op(muffin.OP_PHI, vi.sky.astype(np.float32)).double().cpu().numpy()
    vis = v[..., 0] + 1j * v[..., 1] + vi.noise
    m = muffin.Muffin.from_visibilities(vis, vi.uvw, vi.lam, vi.cell, N=N, J=J, **reg)
    info = m.info()
    print(f"[bench] visibility context ready: beta={info['beta']:.4e} tau={info['tau']:.3e}", file=sys.stderr,
          flush=True)
    if args.autotune:
        m.autotune(reps=3)
    ph = m.profile(args.profile_steps)
    m.step(args.warmup)
    torch.cuda.synchronize()
    dev_ms = m.step_timed(args.steps)
    torch.cuda.synchronize()
    ms_per_step = dev_ms / args.steps
    obj = m.objective()
    m.close()
    vox = N * N * L
    pairs = float(L) * K * N * N  # (visibility, pixel) pairs of one direction
    grad_ms = ph[2]
    achieved = 2 * pairs / (grad_ms * 1e-3)
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms per iteration; phases ms {np.round(ph[:5], 3).tolist()}; "
          f"objective {obj[0]:.6e}", file=sys.stderr, flush=True)
    roof = {
        "bound": "alu",
        "kernel": "visibility gradient (k_vis_fwd + k_vis_adj, with k_vis_xn and k_vis_resid)",
        "achieved": achieved,
        "peak": VIS_PAIR_PEAK,
        "unit": "pairs/s",
        "frac": round(achieved / VIS_PAIR_PEAK, 4),
        "traffic": None,
        "pairs_per_launch": pairs,
        "kernel_avg_ms": round(grad_ms, 4),
        "slots_per_pair": VIS_SLOTS_PER_PAIR,
        "phase_ms": {"adjoint": round(ph[1], 3), "gradient": round(grad_ms, 3), "spectral": round(ph[3], 3),
                     "analysis_dual": round(ph[4], 3)},
    }
    cpu = None
    if not args.no_cpu:
        import tempfile
        Ls = 2
        with tempfile.TemporaryDirectory() as td:
            npz = os.path.join(td, "oracle_vis.npz")
            cv, dt = cpu_baseline_vis(Ls, npz)
            ref = np.load(npz)
            with muffin.Muffin.from_visibilities(ref["vis"], vi.uvw, ref["lam"], vi.cell, N=N, J=J,
                                                 tau=VIS_SAMPLE_TAU, power_iters=2, **reg) as ms:
                ms.set_x(ref["X0"])
                ms.step(1)
                got = {"X": ms.get_x(), "U": ms.get_u(), "V": ms.get_v()}
            err = {k: float(np.linalg.norm(t.double().cpu().numpy() - ref[k]) / np.linalg.norm(ref[k]))
                   for k, t in got.items()}
            err["clipped_fraction_X"] = float(np.mean(ref["X"] == 0))
        print(f"[bench] oracle sample {dt:.1f}s; FP32 vs FP64 errors {err}", file=sys.stderr, flush=True)
        cpu = {"value": cv, "unit": "voxel-iter/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 oracle, the first {Ls} channels of the same inputs ({N}^2, {K} baselines), "
                         f"one iteration from a seeded positive X0 with tau {VIS_SAMPLE_TAU}, {dt:.1f}s "
                         f"single-threaded",
               "fp64_error": {**err, "what": "relative L2 of the GPU's FP32 X, U, V after the same iteration "
                                             "of the same sample"}}
    line = {
        "metric": f"voxel-iterations/s on {N}^2x{L} cube with {K} visibilities per channel "
                  f"(visibility-domain data term, eq. (viseq))",
        "value": vox * args.steps / (dev_ms / 1e3),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"vis{N}_L{L}_K{K}_J{J}", "N": N, "L": L, "K": K, "J": J},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_cnn(args):
    """The warm-start network: inference over the 256 planes of the 1024^2 x 256 cube (the warm start
    of the timed single-cube workload, wall time per cube) and training steps on batches of 16
    planes of 256^2 (forward, backward, Adam)."""
    import torch
    from paper_1602_08847_amd import muffin, synth

    spec = synth.WORKLOADS["cube1024_L256_J5"]
    N, L = spec.N, spec.L
    cube = synth.make_cube(spec, dtype=np.float32, with_sky=False)
    net = muffin.Cnn(seed=1)
    m = muffin.Muffin(cube.dirty, cube.psf, J=spec.J, mu_s=0.25, mu_lambda=3.0)
    del cube
    for _ in range(args.warmup):
        m.warm_start(net)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m.warm_start(net)
    torch.cuda.synchronize()
    ms_inf = (time.perf_counter() - t0) * 1e3 / args.steps
    m.close()
    g = torch.Generator().manual_seed(0)
    x = torch.rand((16, 256, 256), generator=g).cuda()
    y = torch.rand((16, 256, 256), generator=g).cuda()
    for _ in range(args.warmup):
        net.train_step(x, y, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, y, 1e-4)
    torch.cuda.synchronize()
    ms_train = (time.perf_counter() - t0) * 1e3 / args.steps
    net.close()
    # four 3x3 layers 1 -> 32 -> 32 -> 32 -> 1, a multiply-add counted as two flops
    flop_per_px = 2 * 9 * (32 + 32 * 32 + 32 * 32 + 32)
    tflops = flop_per_px * N * N * L / (ms_inf * 1e-3) / 1e12
    line = {
        "metric": "CNN warm start: wall ms per 1024^2x256 cube (inference, normalisation and clamp included)",
        "value": ms_inf,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": False,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "cnn", "planes": L, "N": N, "features": 32, "train_batch": [16, 256, 256]},
        "train_step_ms": ms_train,
        "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tflops / 2500.0, 4), "scope": "whole warm start, all four layers"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

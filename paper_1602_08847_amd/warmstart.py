"""Learned warm start for the MUFFIN iteration: training data, training loop and the
time-to-tolerance comparison against a cold start.

Training pairs are (the warm start's network input, i.e. each dirty channel image divided by its PSF's
main-lobe gain as muffin_warm_input builds it, plain-solver reconstruction of that channel):
seeded synthetic cubes are reconstructed by the library's own primal-dual iteration, and the
network is trained by the library's own forward/backward kernels (muffin_cnn_train_step).  The
comparison runs both starts with identical step sizes against the same reference objective f_ref
(the minimum of a long plain run) and counts iterations and seconds until
(f - f_ref) / |f_ref| <= tol, including the network's inference time for the warm start.

python -m paper_1602_08847_amd.warmstart --help
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import muffin, synth

MU_S, MU_L = 0.25, 3.0


def build_training_set(n_cubes: int, spec: synth.CubeSpec, iters: int, sigma: float, seed0: int = 10000,
                       log=print):
    """Solve n_cubes seeded cubes with the plain iteration; returns GPU tensors (inputs, targets)."""
    import torch
    ins, tgs = [], []
    t0 = time.time()
    for i in range(n_cubes):
        s = synth.CubeSpec(**{**spec.__dict__, "seed": seed0 + i})
        cube = synth.make_cube(s, dtype=np.float32, with_sky=False)
        with muffin.Muffin(cube.dirty, cube.psf, J=s.J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
            ins.append(m.warm_input())  # exactly what muffin_warm_start feeds the network
            m.step(iters)
            tgs.append(m.get_x())
        if log and (i + 1) % max(1, n_cubes // 8) == 0:
            log(f"[warmstart] solved {i + 1}/{n_cubes} training cubes ({time.time() - t0:.1f}s)")
    return torch.cat(ins), torch.cat(tgs)


def build_training_set_batched(n_cubes: int, spec: synth.CubeSpec, iters: int, sigma: float, seed0: int = 10000,
                               group: int = 32, log=print, pool=None, ahead: int = 4):
    """As build_training_set, with ``group`` cubes solved together by the batch API (one graph over
    all their channels); each cube keeps its own step size, so its iterates are those of its own
    context.  Returns GPU tensors (inputs, targets) in seed order.

    ``pool`` (a multiprocessing pool, or None) draws the cubes of the next ``ahead`` groups on the
    host while the GPU solves the current one; the cubes are the same either way."""
    import torch
    ins, tgs = [], []
    t0 = time.time()

    def specs_of(g0):
        return [synth.CubeSpec(**{**spec.__dict__, "seed": seed0 + i}) for i in range(g0, min(n_cubes, g0 + group))]

    pending = {}
    for g0 in range(0, n_cubes, group):
        if pool is not None:
            for g in range(g0, min(n_cubes, g0 + ahead * group), group):
                if g not in pending:
                    pending[g] = [pool.apply_async(synth.make_cube, (s, np.float32, False)) for s in specs_of(g)]
            cubes = [r.get() for r in pending.pop(g0)]
        else:
            cubes = [synth.make_cube(s, dtype=np.float32, with_sky=False) for s in specs_of(g0)]
        with muffin.Batch([(c.dirty, c.psf) for c in cubes], J=spec.J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as b:
            for i in range(len(cubes)):
                ins.append(b.warm_input(i))
            b.step(iters)
            for i in range(len(cubes)):
                tgs.append(b.get_x(i))
        if log:
            log(f"[warmstart] solved {min(n_cubes, g0 + group)}/{n_cubes} training cubes ({time.time() - t0:.1f}s)")
    return torch.cat(ins), torch.cat(tgs)


def train(net: muffin.Cnn, inputs, targets, epochs: int, batch: int, lr: float, seed: int = 0, log=print):
    """Adam on shuffled batches of channel images; returns the per-epoch mean loss.

    An epoch whose mean loss is not below the best so far halves the learning rate, and the
    network ends with the parameters of its best epoch (a late Adam step can throw the loss back
    up by several times)."""
    import torch
    n = inputs.shape[0]
    g = torch.Generator().manual_seed(seed)
    hist = []
    best, best_params = math.inf, None
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tot += net.train_step(inputs[idx].contiguous(), targets[idx].contiguous(), lr)
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if hist[-1] < best:
            best, best_params = hist[-1], net.get_params()
        else:
            lr *= 0.5
        if log:
            log(f"[warmstart] epoch {ep + 1}/{epochs} loss {hist[-1]:.4e} (lr {lr:.2e})")
    if best_params is not None:
        net.set_params(best_params)
    return hist


def time_to_tolerance(m: muffin.Muffin, f_ref: float, tol: float, check_every: int, max_iter: int,
                      trace: list | None = None, trace_every: int = 500):
    """Iterate until (f - f_ref)/|f_ref| <= tol with the library's own stopping rule (muffin_solve,
    objective checked every check_every iterations); returns (iterations, seconds, final f).
    With trace, (iteration, relative gap) pairs are appended every trace_every iterations."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    f = m.objective()[0]
    gap = (f - f_ref) / abs(f_ref)
    if trace is not None:
        trace.append((0, gap))
    while gap > tol and it < max_iter:
        n, f = m.solve(min(trace_every, max_iter - it), check_every=check_every, tol=tol, f_ref=f_ref)
        it += n
        gap = (f - f_ref) / abs(f_ref)
        if trace is not None:
            trace.append((it, gap))
        if it % 20000 < trace_every:
            print(f"[warmstart] {it} iterations, gap {gap:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return it, time.perf_counter() - t0, f


def reference_objective(cube, J: int, sigma: float, iters: int, check_every: int = 100, log=None) -> float:
    """Minimum objective over a long plain run (checked every check_every iterations)."""
    best = math.inf
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        for k in range(iters // check_every):
            m.step(check_every)
            best = min(best, m.objective()[0])
            if log and ((k + 1) * check_every) % 20000 == 0:
                log(f"[warmstart] reference run {(k + 1) * check_every} iterations, f {best:.10e}")
    return best


def reference_run(cube, J: int, sigma: float, iters: int, every: int, tol: float, out_path: str | None = None,
                  log=None) -> dict:
    """A plain run from X = 0 recorded every ``every`` iterations: f_ref is its minimum objective, and
    the same run is the cold start, whose iterations to tol are read from the record (to within
    ``every``).  With out_path the record is rewritten there after every point, so that a run cut
    short keeps what it measured."""
    import torch
    tr = []
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        tr.append((0, float(m.objective()[0])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(every, iters + 1, every):
            m.step(every)
            tr.append((it, float(m.objective()[0])))
            if out_path:
                with open(out_path, "w") as f:
                    json.dump({"every": every, "sigma": sigma, "trace": tr, "s": time.perf_counter() - t0}, f)
            if log and it % 10000 == 0:
                log(f"[warmstart] reference run {it} iterations, f {tr[-1][1]:.10e}")
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
    f_ref = min(f for _, f in tr)
    cross = next((it for it, f in tr if (f - f_ref) / abs(f_ref) <= tol), None)
    return {"f_ref": f_ref, "ref_iters": iters, "ref_every": every, "ref_s": sec, "cold_iters_from_ref": cross,
            "cold_s_from_ref": None if cross is None else sec * cross / iters, "ref_trace": tr, "tol": tol,
            "sigma": sigma, "f0_cold": tr[0][1]}


def compare_cold(cube, J: int, sigma: float, tol: float, f_ref: float, check_every: int, max_iter: int) -> dict:
    """The cold start (X = 0) to the tolerance."""
    out = {"tol": tol, "f_ref": f_ref, "sigma": sigma}
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        out["f0_cold"] = float(m.objective()[0])
        tr = []
        it, sec, f = time_to_tolerance(m, f_ref, tol, check_every, max_iter, tr)
        out.update(cold_iters=it, cold_s=sec, cold_f=f, cold_trace=tr)
    return out


def compare_warm(net: muffin.Cnn, cube, J: int, sigma: float, tol: float, f_ref: float, check_every: int,
                 max_iter: int) -> dict:
    """The warm start (X = max(CNN, 0)) to the tolerance; seconds include the network's inference."""
    import torch
    out = {}
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.warm_start(net)
        torch.cuda.synchronize()
        infer = time.perf_counter() - t0
        out["f0_warm"] = float(m.objective()[0])
        if cube.sky is not None:
            out["snr0_warm_db"] = m.snr(cube.sky)
            inp = np.maximum(m.warm_input().double().cpu().numpy(), 0)
            out["snr_dirty_norm_db"] = float(10 * np.log10(np.sum(cube.sky ** 2) / np.sum((inp - cube.sky) ** 2)))
        tr = []
        it, sec, f = time_to_tolerance(m, f_ref, tol, check_every, max_iter, tr)
        out.update(warm_iters=it, warm_s=sec + infer, warm_infer_s=infer, warm_f=f, warm_trace=tr)
    return out


def compare(net: muffin.Cnn, cube, J: int, sigma: float, tol: float, f_ref: float, check_every: int,
            max_iter: int) -> dict:
    """Cold start (X = 0) against the warm start (X = max(CNN, 0)) on the same cube."""
    out = compare_cold(cube, J, sigma, tol, f_ref, check_every, max_iter)
    out.update(compare_warm(net, cube, J, sigma, tol, f_ref, check_every, max_iter))
    return out


def compare_two_step(cube, J: int, sigma: float, tol: float, f_ref: float, n1: int, check_every: int,
                     max_iter: int) -> dict:
    """The paper's own warm start, its two-step calibration protocol (Sec. 4): n1 iterations with
    mu_lambda = 0 (each channel on its own; the spectral step is skipped), then the full method from
    that X with U = V = 0 until (f - f_ref)/|f_ref| <= tol.  Seconds include both steps."""
    import torch
    out = {"two_step_n1": n1}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=0.0, sigma=sigma) as m1:
        m1.step(n1)
        x1 = m1.get_x()
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        m.set_x(x1)
        out["f0_two_step"] = float(m.objective()[0])
        if cube.sky is not None:
            out["snr0_two_step_db"] = m.snr(cube.sky)
        tr = []
        it, sec, f = time_to_tolerance(m, f_ref, tol, check_every, max_iter, tr)
    out.update(two_step_iters=it, two_step_s=sec + t1, two_step_step1_s=t1, two_step_f=f, two_step_trace=tr)
    return out


def compare_budget(net: muffin.Cnn, cube, J: int, sigma: float, budget: int, check_every: int) -> dict:
    """For cubes where the 1e-4 gap is out of reach in one run: the cold start runs ``budget``
    iterations, and the warm start runs until its objective reaches the cold run's final value
    (at most ``budget`` iterations).  Seconds include the objective checks on both sides and the
    network's inference on the warm side."""
    import torch
    out = {"sigma": sigma, "budget": budget, "check_every": check_every}
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        out["f0_cold"] = float(m.objective()[0])
        tr = [(0, out["f0_cold"])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(check_every, budget + 1, check_every):
            m.step(check_every)
            tr.append((it, float(m.objective()[0])))
            if it % 5000 == 0:
                print(f"[warmstart] cold {it} iterations, f {tr[-1][1]:.6e}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        out.update(cold_iters=budget, cold_s=time.perf_counter() - t0, f_target=tr[-1][1], cold_trace=tr)
    f_target = out["f_target"]
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.warm_start(net)
        torch.cuda.synchronize()
        infer = time.perf_counter() - t0
        f = float(m.objective()[0])
        out["f0_warm"] = f
        tr = [(0, f)]
        it = 0
        while f > f_target and it < budget:
            m.step(check_every)
            it += check_every
            f = float(m.objective()[0])
            tr.append((it, f))
        torch.cuda.synchronize()
        out.update(warm_iters=it, warm_s=time.perf_counter() - t0, warm_infer_s=infer, warm_f=f,
                   warm_reached=bool(f <= f_target), warm_trace=tr)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-cubes", type=int, default=48)
    ap.add_argument("--train-N", type=int, default=256)
    ap.add_argument("--train-L", type=int, default=64)
    ap.add_argument("--train-J", type=int, default=4)
    ap.add_argument("--train-iters", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--sigma", type=float, default=100.0)
    ap.add_argument("--test", default="cube256_L64_J4", help="workload name of the test cube")
    ap.add_argument("--test-seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--ref-iters", type=int, default=20000)
    ap.add_argument("--check-every", type=int, default=20)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--load-params", default=None, help="skip training: load a parameter vector (.npy)")
    ap.add_argument("--net-seeds", default="1",
                    help="comma-separated seeds: one network per seed (initial weights and batch order), each "
                         "trained on the same data and compared against the same cold run")
    ap.add_argument("--two-step", type=int, default=0,
                    help="also run the paper's two-step protocol with this many mu_lambda = 0 iterations first")
    ap.add_argument("--learning-curve", default="",
                    help="comma-separated training-set sizes (cubes): one network per size, trained on the first "
                         "cubes of one batch-solved set, each compared against the same cold run")
    ap.add_argument("--ref-only", action="store_true",
                    help="only the reference run (the cold start, recorded every --ref-every iterations): f_ref and "
                         "the cold start's iterations to --tol, written to --out as it goes")
    ap.add_argument("--ref-every", type=int, default=100)
    ap.add_argument("--f-ref", type=float, default=None,
                    help="f_ref of an earlier reference run: skip the reference and cold runs, run the warm starts")
    ap.add_argument("--autotune", action="store_true", help="tune the band kernels on the test cube first")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="host processes that draw the training cubes while the GPU solves (batch-solved sets)")
    ap.add_argument("--budget", type=int, default=0,
                    help="instead of the 1e-4 gap: iterations of the cold run whose final objective the warm "
                         "start must reach")
    a = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if a.ref_only:
        tspec = synth.WORKLOADS[a.test]
        tspec = synth.CubeSpec(**{**tspec.__dict__, "seed": a.test_seed})
        cube = synth.make_cube(tspec, dtype=np.float32, with_sky=False)
        if a.autotune:
            _tune(cube, tspec.J, a.sigma, log)
        res = reference_run(cube, tspec.J, a.sigma, a.ref_iters, a.ref_every, a.tol,
                            a.out.replace(".json", "_trace.json") if a.out else None, log)
        res.update(test=a.test, test_seed=a.test_seed)
        log(f"[warmstart] f_ref {res['f_ref']:.10e}; cold start within {a.tol} after {res['cold_iters_from_ref']} "
            f"iterations")
        _emit(res, a.out, [])
        return
    spec = synth.CubeSpec(N=a.train_N, L=a.train_L, J=a.train_J, n_sources=20, n_baselines=2000)
    seeds = [int(v) for v in a.net_seeds.split(",")]
    sizes = [int(v) for v in a.learning_curve.split(",")] if a.learning_curve else []
    t_data = 0.0
    inputs = targets = None
    if not a.load_params:
        t0 = time.time()
        n_data = max(sizes) if sizes else a.train_cubes
        if sizes:
            pool = None
            if a.gen_workers > 0:
                import multiprocessing as mp
                # forked before this process first touches the GPU; the workers only run numpy
                pool = mp.get_context("fork").Pool(a.gen_workers)
            try:
                inputs, targets = build_training_set_batched(n_data, spec, a.train_iters, a.sigma, log=log,
                                                             pool=pool)
            finally:
                if pool is not None:
                    pool.terminate()
                    pool.join()
        else:
            inputs, targets = build_training_set(n_data, spec, a.train_iters, a.sigma, log=log)
        t_data = time.time() - t0
    nets = []
    for size in (sizes or [a.train_cubes]):
        for sd in seeds:
            net = muffin.Cnn(seed=sd)
            info = {"net_seed": sd, "train_cubes": size, "loss_hist": [], "t_train_s": 0.0}
            if a.load_params:
                net.set_params(np.load(a.load_params))
            else:
                n_img = size * a.train_L
                # the same number of Adam steps for every size: smaller sets take more epochs
                epochs = a.epochs if not sizes else max(1, round(a.epochs * max(sizes) / size))
                if sizes:
                    epochs = min(epochs, a.epochs * 8)
                info["epochs"] = epochs
                t0 = time.time()
                info["loss_hist"] = train(net, inputs[:n_img], targets[:n_img], epochs, a.batch, a.lr, seed=sd,
                                          log=log)
                info["t_train_s"] = time.time() - t0
            nets.append((net, info))
    del inputs, targets
    tspec = synth.WORKLOADS[a.test]
    tspec = synth.CubeSpec(**{**tspec.__dict__, "seed": a.test_seed})
    cube = synth.make_cube(tspec, dtype=np.float32, with_sky=not a.budget)
    if a.autotune:
        _tune(cube, tspec.J, a.sigma, log)
    common = dict(train_cubes=a.train_cubes, train_iters=a.train_iters, epochs=a.epochs, t_data_s=t_data,
                  test=a.test, test_seed=a.test_seed)
    if a.f_ref is not None:
        res = {**common, "f_ref": a.f_ref, "tol": a.tol, "sigma": a.sigma, "runs": []}
        for net, info in nets:
            w = compare_warm(net, cube, tspec.J, a.sigma, a.tol, a.f_ref, a.check_every, a.max_iter)
            w.update(info)
            log(f"[warmstart] warm (net seed {info['net_seed']}, {info['train_cubes']} training cubes): "
                f"{w['warm_iters']} iterations, {w['warm_s']:.2f}s")
            res["runs"].append(w)
        _emit(res, a.out, nets)
        return
    if a.budget:
        runs = []
        for net, info in nets:
            res = compare_budget(net, cube, tspec.J, a.sigma, a.budget, a.check_every)
            res.update(info)
            runs.append(res)
        _emit({**common, "runs": runs}, a.out, nets)
        return
    t0 = time.time()
    f_ref = reference_objective(cube, tspec.J, a.sigma, a.ref_iters, log=log)
    t_ref = time.time() - t0
    log(f"[warmstart] f_ref {f_ref:.8e} from {a.ref_iters} iterations ({t_ref:.1f}s)")
    res = {**common, "t_ref_s": t_ref, "ref_iters": a.ref_iters}
    res.update(compare_cold(cube, tspec.J, a.sigma, a.tol, f_ref, a.check_every, a.max_iter))
    log(f"[warmstart] cold: {res['cold_iters']} iterations, {res['cold_s']:.2f}s")
    if a.two_step:
        res.update(compare_two_step(cube, tspec.J, a.sigma, a.tol, f_ref, a.two_step, a.check_every, a.max_iter))
        log(f"[warmstart] two-step: {res['two_step_iters']} + {a.two_step} iterations, {res['two_step_s']:.2f}s")
    runs = []
    for net, info in nets:
        w = compare_warm(net, cube, tspec.J, a.sigma, a.tol, f_ref, a.check_every, a.max_iter)
        w.update(info)
        log(f"[warmstart] warm (net seed {info['net_seed']}, {info['train_cubes']} training cubes): "
            f"{w['warm_iters']} iterations, {w['warm_s']:.2f}s")
        runs.append(w)
    res["runs"] = runs
    _emit(res, a.out, nets)


def _tune(cube, J: int, sigma: float, log):
    """The band-height autotuner on the test cube's sizes (its choices hold for the whole process)."""
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=MU_S, mu_lambda=MU_L, sigma=sigma) as m:
        rep = json.loads(m.autotune(reps=3))
    log(f"[warmstart] autotuned: {[(s['j'], s['kernel'], s['rows']) for s in rep['scales']]}, "
        f"fused tail {rep.get('fused_tail')}")


def _emit(res: dict, out: str | None, nets):
    line = json.dumps(res)
    print(line, flush=True)
    if out:
        with open(out, "w") as f:
            f.write(line + "\n")
        for net, info in nets:
            np.save(out.replace(".json", f"_params_n{info['train_cubes']}_seed{info['net_seed']}.npy"),
                    net.get_params())
    for net, _ in nets:
        net.close()


if __name__ == "__main__":
    main()

"""Autotuner of the kernel variants of the FD solver (stfd_tuning).

For a problem shape it times the variants on the GPU and keeps the fastest:

  * the substitution sweeps (step 3 of Algorithm FD, Sec. 4.4): lane-chain
    kernels against matrix-core tile kernels, per right-hand-side count; the
    choice is stored as the smallest count from which the tile kernels win
    (sweep_tile_min_rhs, 0 = never);
  * the band factor (step 3, first half): the panel kernel against the
    streaming one, where no on-chip window kernel applies;
  * the transform GEMMs (steps 2 and 4): workgroup tile height 64 or 128 on
    FP32 matrix cores, 64 x 64, 128 x 64 or 128 x 128 on FP64 ones, and the
    grid order, timed as the full application of the problem's transforms.

Results go to a JSON cache keyed by the shape bucket (precision, padded
half-bandwidth, M_x and N_t rounded to powers of two).  The binding applies
a cached entry right after setup (Problem(..., tuning="cache"), the
default); the cache file is paper_2008_01996_amd/tune_cache.json or the path
in STFD_TUNE_CACHE.

    python -m paper_2008_01996_amd.autotune WORKLOAD [WORKLOAD ...]

(workloads as in bench.py) tunes those shapes on cuda:0 and updates the
cache.  Only timings decide: every variant computes the same mathematics
(the GEMM variants even bit for bit).
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")
CACHE_ENV = "STFD_TUNE_CACHE"
FIELDS = ("sweep_tile_min_rhs", "gemm_tile_m_fp32", "gemm_tile_m_fp64", "gemm_tile_n_fp64", "gemm_n_fast",
          "factor_kernel")
# FP64 GEMM workgroup tiles (rows, columns) the tuner tries
FP64_TILES = ((64, 64), (128, 64), (128, 128))
RHS_COUNTS = (1, 2, 4, 8, 16)


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def _pow2(x: int) -> int:
    return 1 << max(0, int(round(math.log2(max(1, x)))))


def padded_band(half_band: int) -> int:
    return max(16, (half_band + 15) // 16 * 16)


def shape_key(precision: str, Mx: int, half_band: int, Nt: int) -> str:
    """Bucket of a problem shape: precision, padded half-bandwidth, M_x and
    N_t to the nearest power of two."""
    return f"{precision}/bp{padded_band(half_band)}/mx{_pow2(Mx)}/nt{_pow2(Nt)}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data.get("entries", {})


def lookup(entries: dict, precision: str, Mx: int, half_band: int, Nt: int) -> dict | None:
    """The tuning of the shape's bucket; failing that, of the nearest bucket
    (in log2 M_x + log2 N_t) with the same precision and padded band; None
    if there is none."""
    key = shape_key(precision, Mx, half_band, Nt)
    if key in entries:
        return dict(entries[key]["tuning"])
    pre = f"{precision}/bp{padded_band(half_band)}/"
    best, dist = None, None
    for k, e in entries.items():
        if not k.startswith(pre):
            continue
        mx = int(k.split("/mx")[1].split("/")[0])
        nt = int(k.split("/nt")[1])
        d = abs(math.log2(mx) - math.log2(_pow2(Mx))) + abs(math.log2(nt) - math.log2(_pow2(Nt)))
        if dist is None or d < dist:
            best, dist = e, d
    return dict(best["tuning"]) if best else None


def apply(problem, entries: dict | None = None) -> dict | None:
    """Set the cached tuning of the problem's shape (if any) on it; returns
    what was applied."""
    if entries is None:
        entries = load_cache()
    rep = problem.setup_report
    t = lookup(entries, problem.precision, problem.Mx, rep["half_band"], problem.Nt)
    if t:
        t = {k: v for k, v in t.items() if k in FIELDS}
        t.setdefault("gemm_tile_n_fp64", 64)      # entries from before the 128 x 128 tile
        problem.set_tuning(**t)
    return t


# ---------------------------------------------------------------------------
# measurement (GPU)
# ---------------------------------------------------------------------------
def _time(fn, reps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def tune_problem(prob, F, reps: int = 3, rhs_counts=RHS_COUNTS, log=print) -> dict:
    """Time the variants on a set-up problem with device load F (nrhs, N_t,
    M_x); returns {"tuning": ..., "measured": ...}."""
    import torch

    n = prob.setup_report["n_sys"]
    dt = torch.float32 if prob.precision == "fp32" else torch.float64
    measured = {"sweeps_ms": {}, "apply_ms": {}}
    base = prob.tuning()
    # sweeps: chain against tile per right-hand-side count
    wins = []
    for r in rhs_counts:
        G = torch.randn((r, 2 * n, prob.Mx), dtype=dt, device="cuda:0")
        Z = torch.empty_like(G)
        row = {}
        for tile in (0, 1):
            prob.set_tuning(**{**base, "sweep_tile_min_rhs": tile})
            prob.factor()
            row["tile" if tile else "chain"] = _time(lambda: prob.spatial_solve(G, Z), reps)
        measured["sweeps_ms"][str(r)] = row
        wins.append(row["tile"] < row["chain"])
        log(f"  sweeps, {r} RHS: chain {row['chain']:.2f} ms, tile {row['tile']:.2f} ms")
        del G, Z
    tile_min = 0
    for i in range(len(rhs_counts)):
        if all(wins[i:]):
            tile_min = rhs_counts[i]
            break
    # the tile sweeps solve the diagonal blocks through their inverses, which
    # raises the level where the FP32 refinement stalls (by the blocks' Skeel
    # condition); where the workload's own solve is concerned, keep them only
    # if the refined solve converges and is faster with them
    nr = F.shape[0]
    if 0 < tile_min <= nr:
        U = torch.empty_like(F)
        sol = {}
        for tm_ in (tile_min, 0):
            prob.set_tuning(**{**base, "sweep_tile_min_rhs": tm_})
            prob.factor()
            rep = prob.solve(F, U, check=False)
            torch.cuda.synchronize()
            ms = _time(lambda: prob.solve(F, U, check=False), reps) if rep["converged"] else float("inf")
            sol[tm_] = (ms, rep["iterations"], rep["converged"])
            log(f"  refined solve ({nr} RHS), tile sweeps from {tm_ or 'never'}: "
                f"{ms:.2f} ms, {rep['iterations']} applications, converged {rep['converged']}")
        measured["solve_ms"] = {str(k): v[0] for k, v in sol.items()}
        if not sol[tile_min][0] < sol[0][0]:
            tile_min = nr + 1 if nr + 1 <= max(rhs_counts) else 0
    # band factor: the panel kernel against the streaming one (where the
    # automatic choice is not one of the on-chip window kernels)
    bp = padded_band(prob.setup_report["half_band"])
    es = 8 if prob.precision == "fp32" else 16
    window = (prob.precision == "fp32" and bp == 128) or (bp <= 128 and ((bp + 16) * (bp + 1) + 1) * es <= 150 * 1024)
    factor_kernel = 0
    if not window:
        fms = {}
        for fk in ((1, 2, 3) if prob.precision == "fp32" else (1, 2)):
            prob.set_tuning(**{**base, "factor_kernel": fk})
            fms[fk] = _time(prob.factor, reps)
            log(f"  factor kernel {fk}: {fms[fk]:.2f} ms")
        measured["factor_ms"] = {str(k): v for k, v in fms.items()}
        factor_kernel = min(fms, key=fms.get)
    # transforms: one FD application (forward GEMMs, sweeps, back transform)
    X = F
    U = torch.empty_like(F)
    best, best_ms = None, None
    for bm32 in (64, 128):
        for bm64, bn64 in FP64_TILES:
            for nfast in (0, 1):
                t = {"sweep_tile_min_rhs": tile_min, "gemm_tile_m_fp32": bm32, "gemm_tile_m_fp64": bm64,
                     "gemm_tile_n_fp64": bn64, "gemm_n_fast": nfast, "factor_kernel": factor_kernel}
                prob.set_tuning(**t)
                prob.factor()
                ms = _time(lambda: prob.apply(X, U), reps)
                measured["apply_ms"][f"bm32={bm32},fp64 tile={bm64}x{bn64},nfast={nfast}"] = ms
                log(f"  application ({nr} RHS), GEMM tiles {bm32} / {bm64}x{bn64}, n-fast {nfast}: {ms:.2f} ms")
                if best_ms is None or ms < best_ms:
                    best, best_ms = t, ms
    prob.set_tuning(**best)
    prob.factor()
    return {"tuning": best, "measured": measured}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = {"entries": {}}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault("entries", {})[key] = entry
    data["note"] = ("kernel variants of the FD solver per shape bucket, chosen by measured time on one MI355X "
                    "(paper_2008_01996_amd.autotune)")
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


def main(argv) -> None:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    from paper_2008_01996_amd import stfd

    import workloads as wl

    names = argv or [bench.DEFAULT]
    shapes = []
    for name in names:
        if name == "batch96":
            # the nine problem classes of the batch, 8 right-hand sides each
            for nc, nt in sorted({wl.batch_problem_class(p) for p in range(96)}):
                mesh, t = wl.square_mesh(nc), wl.uniform_times(nt)
                modes = [(wl.random_modes(sd), 0) for sd in wl.rhs_seeds("batch", 8, 0)]
                shapes.append((f"batch96 class h=1/{nc} N_t={nt}", mesh, t, modes))
        else:
            spec = bench.WORKLOADS[name]
            shapes.append((name,) + tuple(bench.build_inputs(spec)))
    for name, mesh, t, modes in shapes:
        sp, A, M, Fh = bench.build_loads(mesh, t, modes)
        F = torch.from_numpy(Fh).to("cuda:0")
        for prec in ("fp32", "fp64"):
            # the refined-solve check of the sweep choice runs to half the
            # benchmark's tolerance, so the choice keeps a margin to the level
            # where the FP32 refinement stalls
            prob = stfd.Problem(sp, A, M, precision=prec, tuning=None, rtol=5e-11, max_refine=30)
            key = shape_key(prec, sp.Mx, sp.half_band, len(t) - 1)
            print(f"# tuning {name} {prec} ({key})", flush=True)
            entry = tune_problem(prob, F, log=lambda s: print(s, flush=True))
            entry["workload"] = name
            store(key, entry)
            print(f"# {key}: {entry['tuning']}", flush=True)
            del prob
            torch.cuda.empty_cache()
        del F
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main(sys.argv[1:])

"""Autotuner of the integration launch parameters.

Times integrate_and_bin on a sample of the workload for each candidate of
  integrate_waves_per_cu (0 = one wave per 64-orbit tile, k = persistent grid
  of k waves per CU), integrate_lanes_per_orbit (1 or 2 lanes share an orbit's
  force evaluation) and hist_lds_kb (LDS budget of a histogram workgroup),
keeps the fastest, and caches it per workload shape in a JSON file
($SCHW_TUNE_CACHE, default ~/.cache/schw_tune.json).
"""
import json
import os
import time

from . import _lib as P

CANDIDATES_WAVES = (0, 2, 4, 8)
CANDIDATES_LANES = (1, 2)
CANDIDATES_LDS = (32, 64, 128)


def cache_path():
    return os.environ.get("SCHW_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "schw_tune.json"))


def shape_key(obs, n_pot, n_orb, n_steps, dtype):
    return f"{obs.nx}x{obs.ny}x{obs.nz}|{obs.n_ap}x{obs.nv}|sym{obs.symmetrize}|pots{n_pot}|n{n_orb}|s{n_steps}|{dtype}"


def load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(cfg):
    P.set_tuning("integrate_waves_per_cu", cfg["integrate_waves_per_cu"])
    P.set_tuning("integrate_lanes_per_orbit", cfg.get("integrate_lanes_per_orbit", 1))
    P.set_tuning("hist_lds_kb", cfg["hist_lds_kb"])


def tune(run, key, repeats=2, log=None):
    """run(): one integrate_and_bin call on the sample (synchronised by the caller's
    torch.cuda.synchronize inside).  Returns the best configuration and the table."""
    cache = load_cache()
    if key in cache:
        apply(cache[key]["best"])
        return cache[key]["best"], cache[key]["table"]
    table = []
    for wpc in CANDIDATES_WAVES:
        for lanes in CANDIDATES_LANES:
            for lds in CANDIDATES_LDS:
                cfg = {"integrate_waves_per_cu": wpc, "integrate_lanes_per_orbit": lanes, "hist_lds_kb": lds}
                apply(cfg)
                run()  # warm
                t0 = time.perf_counter()
                for _ in range(repeats):
                    run()
                ms = 1e3 * (time.perf_counter() - t0) / repeats
                table.append(dict(cfg, ms=ms))
                if log:
                    log(f"autotune {cfg}: {ms:.2f} ms")
    best = min(table, key=lambda r: r["ms"])
    best = {k: best[k] for k in ("integrate_waves_per_cu", "integrate_lanes_per_orbit", "hist_lds_kb")}
    apply(best)
    cache[key] = {"best": best, "table": table}
    try:
        os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
        with open(cache_path(), "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return best, table

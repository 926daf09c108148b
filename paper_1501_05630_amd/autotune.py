"""Launch-shape autotuner for the fused sweep-block kernel.

Searches threads per workgroup (then, for a batch of several size classes,
each class's own thread count), cluster moves in flight per workgroup (ICM
slots) and sweeps per launch for one batch of instances (one workgroup per
instance: 64- and 128-thread workgroups let up to 16 small instances share a
compute unit, which pays for batches of many small instances), timing `icm_run` with
HIP events on the context stream, and caches the winner in a JSON file keyed by
the batch's shape.  The choice never changes results: every launch shape
computes the same bits (the random streams are keyed by site, sweep and walker,
not by thread), which the GPU tests check for the shapes the search can pick.
"""
import itertools
import json
import os

THREADS = (64, 128, 256, 512, 1024)
SLOTS = (4, 8, 16, 32)
SWEEPS = (128, 256)


def batch_key(metas, n_instances):
    """Cache key: the distinct unit shapes of the batch (sites, temperatures,
    replicas, cluster-move temperatures, coupling kind) with their counts
    rounded up to a power of two."""
    shapes = {}
    for m in metas:
        k = "N{N}_K{K}_R{R}_Kc{Kc}_j{jkind}".format(**m)
        shapes[k] = shapes.get(k, 0) + 1
    parts = []
    for k in sorted(shapes):
        parts.append(f"{k}x{1 << max(0, (shapes[k] - 1).bit_length())}")
    return "|".join(parts) + f"|n{1 << max(0, (n_instances - 1).bit_length())}"


NO_CLASS_THREADS = [-1, -1, -1, -1]


def candidates(threads=THREADS, slots=SLOTS, sweeps=SWEEPS):
    """Launch shapes the search tries: every combination in which a wave
    carries at most four moves on average (slots <= 4 x waves), the same thread
    count for every size class."""
    out = []
    for t, s, n in itertools.product(threads, slots, sweeps):
        if s > 4 * (t // 64):
            continue
        out.append(dict(threads=t, icm_slots=s, sweeps_per_launch=n, use_graph=1,
                        class_threads=list(NO_CLASS_THREADS)))
    return out


def size_classes(metas):
    """The size classes (as icm_run launches them) present in a batch."""
    return sorted({0 if m["N"] <= 512 else (1 if m["N"] <= 1024 else (2 if m["N"] <= 2048 else 3))
                   for m in metas})


def event_timer(ctx, handles, sweeps, repeats=2):
    """ms per sweep of icm_run over `handles`, by HIP events on the context
    stream, after one untimed run (which also captures the launch graph)."""
    torch = ctx.torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.icm_run(handles, sweeps)
    ctx.icm_sync()
    e0.record(ctx.stream)
    for _ in range(repeats):
        ctx.icm_run(handles, sweeps)
    e1.record(ctx.stream)
    ctx.icm_sync()
    return e0.elapsed_time(e1) / (repeats * sweeps)


def _load(cache_path):
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _store(cache_path, cache):
    if not cache_path:
        return
    d = os.path.dirname(cache_path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)


def tune(ctx, handles, cache_path=None, cands=None, sweeps_per_candidate=None, timer=event_timer,
         verbose=False):
    """Picks the fastest launch shape for this batch, applies it to ctx and
    returns (config, info).  info: the cache key, where the choice came from
    ("cache" or "search") and, after a search, each candidate's ms per sweep.

    A search runs every candidate on the live instances, so their state
    advances: tune on a warm-up batch, or reset the states afterwards."""
    key = batch_key([ctx.meta[h] for h in handles], len(handles))
    cache = _load(cache_path)
    if key in cache:
        best = dict(cache[key])
        best["class_threads"] = list(best.get("class_threads", NO_CLASS_THREADS))
        ctx.icm_set_run_config(**best)
        return best, {"key": key, "source": "cache"}
    results = []
    for cfg in (cands if cands is not None else candidates()):
        cfg = dict(cfg, class_threads=list(cfg.get("class_threads", NO_CLASS_THREADS)))
        ctx.icm_set_run_config(**cfg)
        n = sweeps_per_candidate or cfg["sweeps_per_launch"]
        ms = timer(ctx, handles, n)
        results.append((ms, cfg))
        if verbose:
            print(f"autotune {key} {cfg}: {ms * 1e3:.2f} us/sweep", flush=True)
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    # a batch of several size classes (one launch each): then each class's
    # thread count is refined in turn, the others held, on the whole batch
    classes = size_classes([ctx.meta[h] for h in handles])
    if len(classes) > 1:
        best_ms = results[0][0]
        ct = list(NO_CLASS_THREADS)
        for cls in classes:
            for t in THREADS:
                trial = list(ct)
                trial[cls] = t
                cfg = dict(best, class_threads=list(trial))
                ctx.icm_set_run_config(**cfg)
                ms = timer(ctx, handles, sweeps_per_candidate or cfg["sweeps_per_launch"])
                results.append((ms, cfg))
                if verbose:
                    print(f"autotune {key} {cfg}: {ms * 1e3:.2f} us/sweep", flush=True)
                if ms < best_ms:
                    best_ms, ct = ms, trial
        best["class_threads"] = list(ct)
    cache[key] = best
    _store(cache_path, cache)
    ctx.icm_set_run_config(**best)
    return best, {"key": key, "source": "search",
                  "ms_per_sweep": {json.dumps(c, sort_keys=True): ms for ms, c in results}}

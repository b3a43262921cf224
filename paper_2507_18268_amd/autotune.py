"""Autotuner for the batched form and the serving loop.

Batched form: for each bucket (cube side range) a set of synthetic problems of
that size is solved by the persistent batched kernel with every candidate
workgroup size, and the size with the highest throughput (cells x steps per
second of device time) is kept.

Serving loop: a short stream of synthetic requests (sides log-uniform in
[16, 96], all arriving at once) is served with every candidate pair of lane
threshold (the smallest cube side that leaves the batched kernel for the
multi-kernel solver) and inner iterations per group workgroup, and the pair
with the most solves per second is kept.

Results are cached in a JSON file keyed by the GPU architecture and the form,
so the choice is stable from run to run (a problem's result depends on the
workgroup size and on its lane, so a fixed table also keeps results
reproducible).
"""
import json
import os
import time

from . import lapfoam as L

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
CANDIDATES = (256, 512, 1024)
# serving: lane threshold (cube side) and inner iterations per group workgroup
LANE_CANDIDATES = (16, 20, 24, 32, 40)
GROUP_ITERS_CANDIDATES = (1, 2, 4)
# what the serving loop uses when nothing is cached
SERVING_DEFAULT = {"direct_min_side": 24, "group_iters": 2}
# (lower side, upper side) of each bucket and the side used to measure it
BUCKETS = ((0, 20, 16), (20, 28, 24), (28, 40, 32), (40, 56, 48), (56, 76, 64), (76, 1 << 30, 96))


def arch_key():
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def bucket_of(side):
    for i, (lo, hi, _) in enumerate(BUCKETS):
        if lo <= side < hi:
            return i
    return len(BUCKETS) - 1


def load(path=CACHE, form="mixed"):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    return data.get(f"{arch_key()}/{form}")


def serving_params(path=CACHE):
    """The serving loop's lane threshold and group iterations: the cached
    choice for this architecture, else SERVING_DEFAULT."""
    t = load(path, "serving")
    if not t:
        return dict(SERVING_DEFAULT)
    return {"direct_min_side": int(t["direct_min_side"]), "group_iters": int(t["group_iters"])}


def block_threads_for(side, table=None, default=512):
    table = table if table is not None else load()
    if not table:
        return default
    return int(table["block_threads"][bucket_of(side)])


def measure(side, bs, copies=64, steps=3, seed=0):
    """Device time per launch of `copies` problems of one side, in seconds."""
    import torch
    import synth
    mesh = synth.box_mesh(side, side, side)
    m = L.Mesh(mesh)
    probs = []
    for i in range(copies):
        # the layout the server gives batched requests: bands on 3-band meshes
        lay = L.LF_LAYOUT_AUTO if m.n_bands == 3 else L.LF_LAYOUT_ROWS
        P = L.Problem(m, synth.fixed_x_bcs(), 1e-3 * (1 + i % 7), 1e-3,
                      L.make_opts(precision=L.LF_PREC_MIXED, layout=lay))
        P.set_T(synth.initial_field(mesh.n_cells, seed + i))
        probs.append(P)
    b = L.Batch(copies, steps)
    torch.cuda.synchronize()
    b.launch(probs, steps, block_threads=bs)      # warm-up
    b.wait()
    for i, P in enumerate(probs):
        P.set_T(synth.initial_field(mesh.n_cells, seed + i))
    torch.cuda.synchronize()
    b.launch(probs, steps, block_threads=bs)
    b.wait()
    _, ms = b.stats()
    for P in probs:
        P.close()
    b.close()
    m.close()
    return ms * 1e-3, mesh.n_cells * copies * steps


def _store(form, table, path, out_path):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[f"{arch_key()}/{form}"] = table
    with open(out_path or path, "w") as f:
        json.dump(data, f, indent=1)


def measure_serving(direct_min_side, group_iters, n_requests=256, seed=0x5E41, workers=32, passes=3):
    """Saturated solves per second of one serving loop over n_requests requests
    (all arriving at once): the median of `passes` passes after one warm-up
    pass over the same stream."""
    import torch
    import synth
    from . import serve as S
    meshes = {}

    def mesh_for_side(n):
        if n not in meshes:
            meshes[n] = synth.box_mesh(n, n, n)
        return meshes[n]

    stream = synth.request_stream(n_requests, rate=1.0, seed=seed)
    srv = S.Server(mesh_for_side, 64 << 30, max_steps=10, direct_min_side=direct_min_side,
                   direct_workers=workers, group_iters=group_iters)
    for n in sorted({r.n for r in stream}):
        srv.preload_mesh(n)
    torch.cuda.synchronize()
    rates = []
    for _ in range(1 + passes):
        reqs = [S.Request(rid=r.rid, n=r.n, DT=r.DT, dt=r.dt, steps=r.steps,
                          T0=synth.initial_field(r.n ** 3, r.seed), bcs=synth.fixed_x_bcs(),
                          arrival=0.0) for r in stream]
        done = srv.run(reqs, poll_s=0.0)
        ok = len(done) == len(reqs) and all(all(s["converged"] == 1 for s in r.stats) for r in done)
        rates.append(S.summarize(done)["solves_per_s"] if ok else 0.0)
    srv.close()
    return 0.0 if 0.0 in rates else sorted(rates[1:])[len(rates[1:]) // 2]


def tune_serving(path=CACHE, n_requests=256, verbose=True, out_path=None):
    """Pick the lane threshold and group iterations with the most saturated
    solves per second; a run that loses a request or leaves one unconverged
    scores zero."""
    table = {"lane_candidates": list(LANE_CANDIDATES),
             "group_iters_candidates": list(GROUP_ITERS_CANDIDATES),
             "n_requests": n_requests, "solves_per_s": {},
             "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    best, best_rate = None, -1.0
    for side in LANE_CANDIDATES:
        for it in GROUP_ITERS_CANDIDATES:
            rate = measure_serving(side, it, n_requests=n_requests)
            table["solves_per_s"][f"{side}/{it}"] = rate
            if verbose:
                print(f"[autotune] serving lane >= {side}, {it} iterations per block: "
                      f"{rate:.1f} solves/s", flush=True)
            if rate > best_rate:
                best, best_rate = (side, it), rate
    table["direct_min_side"], table["group_iters"] = best
    _store("serving", table, path, out_path)
    return table


def tune(path=CACHE, copies=64, steps=3, verbose=True, out_path=None):
    table = {"block_threads": [], "throughput": [], "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    for lo, hi, side in BUCKETS:
        best, best_rate, rates = None, -1.0, {}
        for bs in CANDIDATES:
            sec, work = measure(side, bs, copies=copies, steps=steps)
            rate = work / sec
            rates[bs] = rate
            if rate > best_rate:
                best, best_rate = bs, rate
        table["block_threads"].append(best)
        table["throughput"].append({str(k): v for k, v in rates.items()})
        if verbose:
            print(f"[autotune] side {side}: " + ", ".join(f"{k}: {v:.3g} cell-steps/s"
                                                          for k, v in rates.items()) + f" -> {best}",
                  flush=True)
    _store("mixed", table, path, out_path)
    return table


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--form", choices=("mixed", "serving", "all"), default="all")
    ap.add_argument("--out", default=None, help="write the cache here instead of in place")
    a = ap.parse_args()
    if a.form in ("mixed", "all"):
        tune(out_path=a.out)
    if a.form in ("serving", "all"):
        tune_serving(path=a.out or CACHE, out_path=a.out)

"""Autotuner for the batched form: workgroup size per mesh-size bucket.

For each bucket (cube side range) a set of synthetic problems of that size is
solved by the persistent batched kernel with every candidate workgroup size,
and the size with the highest throughput (cells x steps per second of device
time) is kept.  Results are cached in a JSON file keyed by the GPU
architecture and the precision form, so the choice is stable from run to run
(a problem's result depends on the workgroup size, so a fixed table also keeps
results reproducible).
"""
import json
import os
import time

from . import lapfoam as L

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
CANDIDATES = (256, 512, 1024)
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


def load(path=CACHE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    return data.get(f"{arch_key()}/mixed")


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
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[f"{arch_key()}/mixed"] = table
    with open(out_path or path, "w") as f:
        json.dump(data, f, indent=1)
    return table


if __name__ == "__main__":
    import sys
    tune(out_path=sys.argv[1] if len(sys.argv) > 1 else None)

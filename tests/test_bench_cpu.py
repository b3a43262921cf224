"""The benchmark's algorithmic byte counts (no GPU): the per-unit figures the
roofline objects divide by."""
import bench


def test_gradient_bytes_per_launch():
    n = 256
    N, F, B = n ** 3, 3 * n * n * (n - 1), 6 * n * n
    # band path: 44 B per cell, 32 B per band slot (3 per cell), 76 B per boundary face
    assert bench.grad_bytes(N, F, B, 3) == 44 * N + 96 * N + 76 * B == 2378694656
    # row path: 45 B per cell, 72 B per internal face, 76 B per boundary face (+24 B per cell reordered)
    assert bench.grad_bytes(N, F, B) == 45 * N + 72 * F + 76 * B
    assert bench.grad_bytes(N, F, B, 0, True) - bench.grad_bytes(N, F, B) == 24 * N
    # as the corrected step runs it: no snGrad_b and no boundary gradient (44 B per boundary face)
    assert bench.grad_bytes(N, F, B, 3, boundary_gradient=False) == 44 * N + 96 * N + 44 * B
    assert bench.grad_bytes(N, F, B, boundary_gradient=False) == 45 * N + 72 * F + 44 * B


def test_amul_bytes_per_launch():
    n = 256
    N, F = n ** 3, 3 * n * n * (n - 1)
    assert bench.amul_bytes(N, F) == 24 * N + 16 * F == 1204813824


def test_gpus_other_than_one_are_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout


def test_serving_parameters_from_the_cache(tmp_path, monkeypatch):
    """The serving loop's lane threshold and group iterations come from the
    autotuner's cache for this architecture, else from the stated default."""
    import json
    from paper_2507_18268_amd import autotune
    monkeypatch.setattr(autotune, "arch_key", lambda: "gfx950")
    path = str(tmp_path / "cache.json")
    assert autotune.serving_params(path) == autotune.SERVING_DEFAULT
    with open(path, "w") as f:
        json.dump({"gfx942/serving": {"direct_min_side": 40, "group_iters": 4}}, f)
    assert autotune.serving_params(path) == autotune.SERVING_DEFAULT     # another GPU's
    with open(path, "w") as f:
        json.dump({"gfx950/serving": {"direct_min_side": 20, "group_iters": 1}}, f)
    assert autotune.serving_params(path) == {"direct_min_side": 20, "group_iters": 1}
    autotune._store("mixed", {"block_threads": [512] * len(autotune.BUCKETS)}, path, None)
    with open(path) as f:
        data = json.load(f)
    assert set(data) == {"gfx950/serving", "gfx950/mixed"}                 # one form kept beside the other

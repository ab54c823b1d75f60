"""Host-side checks that need no GPU: the bench's self-checks (backward errors)
detect wrong solutions, the bench refuses more than one GPU, and the product
code never reaches the oracle (only the tests, smoke() and the bench's CPU
baseline may)."""
import ast
import os
import subprocess
import sys

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def _dense(a, b, c, periodic):
    n = b.size
    A = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    if periodic:
        A[0, -1] += a[0]
        A[-1, 0] += c[-1]
    return A


def test_line_residual_accepts_solutions_and_rejects_perturbed_ones():
    bench = _bench()
    rng = np.random.default_rng(3)
    for periodic in (False, True):
        a, b, c = W.random_tridiag(40, rng, periodic=periodic)
        d = rng.standard_normal((6, 40))
        x = np.linalg.solve(_dense(a, b, c, periodic), d.T).T
        assert bench.line_residual(a, b, c, x, d, periodic) < 1e-15
        x[3, 17] *= 1 + 1e-9
        assert bench.line_residual(a, b, c, x, d, periodic) > 1e-11


def test_apply_tri_composes_along_axes():
    """A_z A_y A_x applied along three axes equals the Kronecker-structured product."""
    bench = _bench()
    rng = np.random.default_rng(4)
    u = rng.standard_normal((5, 4, 6))
    cx, cy, cz = W.momentum_uniform(6), W.momentum_stretched(4), W.momentum_periodic(5)
    y = u
    for (a, b, c), axis, per in ((cz, 0, True), (cy, 1, False), (cx, 2, False)):
        y, _ = bench.apply_tri(a, b, c, y, axis, per)
    want = np.einsum("ai,bj,ck,ijk->abc", _dense(*cz, True), _dense(*cy, False), _dense(*cx, False), u)
    assert np.max(np.abs(y - want)) < 1e-12 * np.max(np.abs(want))


def test_poisson_rows_pin_the_zero_mode():
    bench = _bench()
    ay, cy = W.poisson_metric(16)
    lam = W.modified_wavenumbers(8)
    a, b, c, pin = bench.poisson_rows(ay, cy, lam)
    assert pin[0] and not pin[1:].any()
    assert b[0, 0] == 1.0 and c[0, 0] == 0.0 and a[0, 0] == 0.0
    assert np.array_equal(b[1], -(ay + cy) - lam[1])


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _imports(path):
    tree = ast.parse(open(path).read())
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module:
            names.add(node.module.split(".")[0])
    return names


def test_product_code_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1812_01178_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                assert "oracle" not in _imports(os.path.join(dirpath, f)), f
    for f in os.listdir(os.path.join(ROOT, "workloads")):
        if f.endswith(".py"):
            assert "oracle" not in _imports(os.path.join(ROOT, "workloads", f)), f
    # bench.py: only inside the CPU-baseline block of main()
    src = open(os.path.join(ROOT, "bench.py")).read().splitlines()
    uses = [i for i, ln in enumerate(src) if "import oracle" in ln or "from oracle" in ln]
    assert len(uses) == 1 and "cpu_baseline" in src[uses[0] + 1]


def test_spikes_of_dominant_blocks_sum_to_at_most_one():
    """The shifted Poisson solves eliminate the reduced system without pivoting
    because, for a row-dominant block, the left and right spikes satisfy
    |v_j| + |w_j| <= 1 at every row (maximum principle: they are the block's
    response to unit boundary values).  Checked on random dominant blocks and on
    the weakly dominant Neumann-metric rows with zero shift, whose bound is tight."""
    rng = np.random.default_rng(12)

    def spikes(a, b, c):
        m = b.size
        B = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        e0 = np.zeros(m); e0[0] = a[0]
        em = np.zeros(m); em[-1] = c[-1]
        return np.linalg.solve(B, e0), np.linalg.solve(B, em)

    for _ in range(200):
        m = int(rng.integers(2, 33))
        a, b, c = W.random_tridiag(m, rng, periodic=True, margin=float(rng.uniform(0.0, 2.0)))
        v, w = spikes(a, b, c)
        assert np.max(np.abs(v) + np.abs(w)) <= 1.0 + 1e-12
    ay, cy = W.poisson_metric(256)
    for sigma in (0.0, 1e-3, 39.5):
        for lo, m in ((32, 32), (96, 16), (224, 32)):
            sl = slice(lo, lo + m)
            v, w = spikes(ay[sl], -(ay[sl] + cy[sl]) - sigma, cy[sl])
            s = np.abs(v) + np.abs(w)
            assert np.max(s) <= 1.0 + 1e-12
            if sigma == 0.0 and lo + m < 256:
                assert np.max(s) > 1.0 - 1e-9       # tight: constants solve the homogeneous rows


def test_bench_oracle_parity_scores_every_kept_result(orc):
    """bench.py's CPU-baseline leg compares every kept pristine-input result with
    the oracle: results equal to the oracle's score 0, and one perturbed entry
    anywhere in a field shows up in that solve's worst-line error."""
    bench = _bench()
    nz, ny, nx = 288, 32, 64                 # spanwise lines of the benchmark: PDD at P = 16 is exact there
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal((nz, ny, nx))
    phi0 = rng.standard_normal((nz // 2 + 1, ny, nx)) + 1j * rng.standard_normal((nz // 2 + 1, ny, nx))
    coef = {"x": W.momentum_uniform(nx), "y": W.momentum_stretched(ny), "z": W.momentum_periodic(nz)}
    ay, cy = W.poisson_metric(ny)
    lam = W.modified_wavenumbers(nz)

    def results(ld):
        out = {}
        for name, d, P, per, _ in bench.ITEMS:
            if name == "poisson":
                ref = phi0.copy()
                orc.poisson(ref, ay, cy, lam, P=P, method=orc.EXACT_LD if ld else orc.PPT)
            else:
                ref = u0.copy()
                orc.adi_sweep(orc.EXACT_LD if ld else orc.PDD, d, ref, *coef["xyz"[d]], P, per)
            out[name] = ref
        return out

    u_keep, phi_keep = u0.copy(), phi0.copy()
    pristine = {"fp64": results(False), "fp32_refine": results(True)}
    pristine["fp64"]["adi_y"][5, 7, 9] += 1e-9 * np.max(np.abs(pristine["fp64"]["adi_y"]))
    err = bench.oracle_parity(orc, pristine, u0, phi0, coef, ay, cy, lam)
    assert err["fp64"]["adi_x"] == 0 and err["fp64"]["adi_z"] == 0 and err["fp64"]["poisson"] == 0
    assert err["fp64"]["adi_y"] > 1e-10
    # the exact solutions are within round-off of the FP64 oracle's solves on these rows
    assert max(err["fp32_refine"].values()) < 1e-13
    assert np.array_equal(u0, u_keep) and np.array_equal(phi0, phi_keep)    # inputs left as they were


def test_bench_cpu_baseline_leaves_its_inputs_untouched(orc):
    bench = _bench()
    nz, ny, nx = 288, 32, 64
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal((nz, ny, nx))
    phi0 = rng.standard_normal((nz // 2 + 1, ny, nx)) + 1j * rng.standard_normal((nz // 2 + 1, ny, nx))
    keep_u, keep_p = u0.copy(), phi0.copy()
    coef = {"x": W.momentum_uniform(nx), "y": W.momentum_stretched(ny), "z": W.momentum_periodic(nz)}
    ay, cy = W.poisson_metric(ny)
    bench.cpu_baseline(orc, u0, phi0, coef, ay, cy, W.modified_wavenumbers(nz), 0.01)
    assert np.array_equal(u0, keep_u) and np.array_equal(phi0, keep_p)


def test_tune_table_lists_the_ragged_partition_choices():
    """The shipped tuning table fixes the partition count of every item of the
    ragged eight-sub-grid batch (x, y, z sweeps and Poisson, FP64 and FP32+refine,
    and FP64 with the levels as level launches), so every run of the benchmark
    measures the same configuration."""
    table = open(os.path.join(ROOT, "paper_1812_01178_amd", "tune_gfx950.txt")).read().splitlines()
    keys = {ln.rsplit("|", 1)[0]: int(ln.rsplit("|", 1)[1]) for ln in table if "|" in ln and not ln.startswith("#")}
    for prec, suffix in ((0, ""), (1, ""), (0, " L")):     # " L": the FP64 plan's level launches
        for nx, ny, nz in W.RAGGED_SUBGRIDS:
            for kind, per, method, n3 in ((0, 0, 0, nz), (1, 0, 0, nz), (2, 1, 0, nz), (3, 0, 1, nz // 2 + 1)):
                key = f"partitions k{kind} m{method} per{per} prec{prec} Nx{nx} Ny{ny} Nz{n3}{suffix}"
                assert keys.get(key, 0) in (1, 2, 4, 8, 16), key

"""Model shapes used by the tests and the bench, with matching oracle models.

Shapes follow the workloads: the tiny Gaussian-blob fit (8 levels, growth
1.5 from 4, 2^14 entries, 16-32-32-1), the inference/training model (16
levels from 16 to 2048, 2^19 entries, 32-64-64-1), the paper's fixed
Table-2 network (8 levels x 8 features, 2^19, 64 wide, 4 hidden), a
4-feature variant, a 32-level narrow model, a 4-level model with large
tables (fewer levels than XCDs), a 12-level model (level pairs of the
level-split query that hold one level), and 8- and 12-level models whose
levels all fit LDS over a brick (one level per XCD group; every level pair
shared by all XCDs).
"""
import numpy as np

import oracle
import synth

SEED = 2207_11620

MODELS = {
    "tiny": dict(L=8, F=2, log2T=14, base=4, scale=1.5, maxres=0, width=32, n_hidden=2, table_scale=1e-4),
    "cfg1": dict(L=16, F=2, log2T=19, base=16, scale=0.0, maxres=2048, width=64, n_hidden=2, table_scale=1e-2),
    "paper": dict(L=8, F=8, log2T=19, base=4, scale=2.0, maxres=0, width=64, n_hidden=4, table_scale=1e-4),
    "f4": dict(L=16, F=4, log2T=16, base=16, scale=0.0, maxres=1024, width=64, n_hidden=2, table_scale=1e-2),
    "w32k64": dict(L=32, F=2, log2T=12, base=4, scale=1.2, maxres=0, width=32, n_hidden=3, table_scale=1e-2),
    "l4": dict(L=4, F=2, log2T=20, base=64, scale=0.0, maxres=1024, width=32, n_hidden=1, table_scale=1e-2),
    "l12": dict(L=12, F=2, log2T=19, base=16, scale=0.0, maxres=1024, width=64, n_hidden=2, table_scale=1e-2),
    "l8s": dict(L=8, F=2, log2T=19, base=16, scale=0.0, maxres=256, width=64, n_hidden=2, table_scale=1e-2),
    "l12s": dict(L=12, F=2, log2T=19, base=16, scale=0.0, maxres=256, width=64, n_hidden=2, table_scale=1e-2),
}


def oracle_model(name, out_relu=False):
    c = MODELS[name]
    res = oracle.resolutions(c["L"], c["base"], c["scale"], c["maxres"])
    return oracle.Model(c["L"], c["F"], c["log2T"], res, c["width"], c["n_hidden"], out_relu=out_relu)


def gpu_plan(name, precision="fp32", loss="l2", out_relu=False):
    import paper_2207_11620_amd as ngv
    c = MODELS[name]
    return ngv.Plan(c["L"], c["F"], c["log2T"], c["base"], c["scale"] or 2.0, c["maxres"], n_neurons=c["width"],
                    n_hidden_layers=c["n_hidden"], precision=precision, loss=loss,
                    output_activation="relu" if out_relu else "none")


def init_params(name, seed=SEED, table_scale=None):
    c = MODELS[name]
    m = oracle_model(name)
    ts = c["table_scale"] if table_scale is None else table_scale
    return synth.init_params(m.n_table, m.n_in, c["width"], c["n_hidden"], ts, seed)


def rel_err(got, ref):
    """Normwise relative error max|got-ref| / max|ref|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (den if den > 0 else 1.0))


def edge_coords(n, seed=5):
    """Random coordinates with the edge cases in front: corners, x = 1, outside
    the cube (clamped) and NaN (treated as 0)."""
    xyz = synth.rng_u01(seed, synth.STREAM_QUERY, np.arange(3 * n)).reshape(n, 3).copy()
    edge = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0.5], [0.5, 0.5, 0.5], [-0.2, 1.3, 0.7], [np.nan, 0.25, 0.75],
                     [0.9999999, 1e-8, 0.5], [0.25, 0.5, 0.75]], np.float32)
    xyz[:len(edge)] = edge
    return np.ascontiguousarray(xyz)

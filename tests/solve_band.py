"""After-solve gates for chaotic CGLS workloads, from the band the FP64
oracle's own solve spans when every operator application is perturbed by a
relative L2 amount of the size of a GPU precision's rounding
(tests/golden/solve_spread.json, written by tests/golden/make_solve_spread.py,
which calls only the oracle).

On several workloads CG turns a change in the 13th digit of one application
into a 1e-3 .. 1e-2 change of the final F and iterate: the oracle re-run with
nothing but its inner products summed in another order lands that far from
itself.  A GPU solve rounds differently in every application, so after the
solve it is held to the larger of the fixed target and FACTOR times the
largest change measured over the oracle's perturbed solves (three seeds):
  * PA_F64 against the f64 band (eps 1e-13);
  * PA_MIXED and PA_F32 against the f32 band (eps 1e-6: FP32 delays and
    weights).
"""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
FACTOR = 3.0
_data = None


def band(case: str, precision: str) -> dict:
    """precision: "f64", "mixed" or "f32" (the last two share the f32 band)."""
    global _data
    if _data is None:
        with open(os.path.join(HERE, "golden", "solve_spread.json")) as f:
            _data = json.load(f)
    return _data[case]["f64" if precision == "f64" else "f32"]


def gates(case: str, precision: str, target: float = 1e-4) -> dict:
    """Gates on the final iterate (relative L2), F_N and ||r_N|| (relative)."""
    b = band(case, precision)
    g = {"x": max(target, FACTOR * b["x_rel_l2"]),
         "F": max(target, FACTOR * b["F_rel_by_k"][-1]),
         "r": max(target, FACTOR * b["r_rel_by_k"][-1])}
    if "x_sample_rel_l2" in b:
        g["x_sample"] = max(target, FACTOR * b["x_sample_rel_l2"])
    return g

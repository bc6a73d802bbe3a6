"""The paper's linear elastostatics benchmark (Sec. 5.1.2) on the GPU.

Manufactured solution on the unit cube, Young's modulus E = cos(m pi x y z) + 2,
solved by V-cycles on the 6-macro Kuhn cube at levels 3..5 (the paper's
levels 1..3) with errors measured on level 6.  Checks: second-order
convergence of the physically scaled operator (row-wise interface rule, as
the paper runs it), errors within a factor 2 of the values the paper prints
(tests/golden/elastostatics_errors.json, its Table tab:benchmarkphysical_and_
unphysical), and the stagnation of the unphysical scaling."""
import json
import os

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "elastostatics_errors.json")))


def test_physical_scaling_converges_at_second_order():
    from paper_1908_08666_amd import elastostatics as E
    variants = {"physical": dict(corr="physical", op_method="scaled"),
                "unphysical": dict(corr="none", op_method="scaled")}
    res = E.benchmark([3, 4, 5], 6, ms=(1,), variants=variants)
    phys, unph = res["m1_physical"], res["m1_unphysical"]
    for r in phys + unph:
        print(f"  {r}", flush=True)
        assert r["status"] == "HHG_OK" and r["iterations"] <= 40
    assert phys[1]["eoc"] >= 1.8 and phys[2]["eoc"] >= 1.7
    for q, paper in enumerate(GOLD["physical"]["1"][:2]):
        assert 0.5 <= phys[q]["error"] / paper <= 2.0, (phys[q]["error"], paper)
    # without the correction the error stalls at the scaling's inconsistency
    assert unph[2]["error"] >= 5.0 * phys[2]["error"]
    assert unph[2]["eoc"] <= 0.5


def test_fp32_cycles_keep_the_discretisation_error():
    """V-cycles in FP32 inside the FP64 V-cycle iteration reach the same
    discrete solution: the errors against u* agree with those of FP64 cycles
    to far below the discretisation error (the algebraic error at the
    stopping tolerance 1e-8 is what separates them)."""
    from paper_1908_08666_amd import elastostatics as E
    variants = {"f64": dict(corr="physical", op_method="scaled"),
                "f32": dict(corr="physical", op_method="scaled", precision="f32")}
    res = E.benchmark([3, 4, 5], 6, ms=(8,), variants=variants)
    for a, b in zip(res["m8_f64"], res["m8_f32"]):
        print(f"  level {a['level']}: FP64 cycles {a['error']:.6e} ({a['iterations']} it), "
              f"FP32 cycles {b['error']:.6e} ({b['iterations']} it)", flush=True)
        assert b["status"] == "HHG_OK" and b["iterations"] <= a["iterations"] + 2
        assert abs(b["error"] - a["error"]) <= 1e-4 * a["error"]


def test_zerosum_rule_keeps_second_order_under_cg():
    """A symmetric operator with second-order accuracy at the interfaces: the
    zero-sum interface centre solved by V-cycle CG converges like the
    row-wise rule (m = 8, where the nodal centre of the symmetric rule falls
    below first order), with errors within 10 % of the row-wise ones."""
    from paper_1908_08666_amd import elastostatics as E
    variants = {"rowwise": dict(corr="physical", op_method="scaled", iface="rowwise", method="cycle"),
                "zerosum": dict(corr="physical", op_method="scaled", iface="zerosum", method="cg"),
                "symmetric": dict(corr="physical", op_method="scaled", iface="symmetric", method="cg")}
    res = E.benchmark([3, 4, 5], 6, ms=(8,), variants=variants)
    for name in variants:
        for r in res[f"m8_{name}"]:
            print(f"  {name}: {r}", flush=True)
            assert r["status"] == "HHG_OK"
    zs, rw, sy = res["m8_zerosum"], res["m8_rowwise"], res["m8_symmetric"]
    assert zs[1]["eoc"] >= 1.8 and zs[2]["eoc"] >= 1.7
    assert sy[2]["eoc"] < 1.0
    for a, b in zip(zs, rw):
        assert abs(a["error"] / b["error"] - 1) <= 0.1
    assert all(r["iterations"] <= 20 for r in zs)

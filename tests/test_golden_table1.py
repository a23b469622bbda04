"""Table 1 (ensemble parameters) and the sec. 2.3 overlap parameters, as
transcribed in tests/golden/table1_ensembles.json, against the synthetic
workloads that stand in for the ensembles: same shapes, masses, clover
coefficient, twist and kernel parameter."""
import json
import os

import bench

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "table1_ensembles.json")) as f:
        return json.load(f)


def test_twisted_clover_workload_is_milc12():
    t = _golden()["MILC12"]
    assert bench.TM_LAT == (t["L"], t["L"], t["L"], t["T"])
    assert bench.M == t["m_wilson"] and bench.CSW == t["c_sw"]


def test_hisq_workload_is_milc09_shape():
    t = _golden()["MILC09"]
    assert bench.HISQ_LAT == (t["L"], t["L"], t["L"], t["T"])
    # the 8 masses bracket the Table 3 light masses of both ensembles
    h = _golden()["_table3"]
    assert min(bench.HISQ_MASSES) < h["MILC09_hisq_mass"] < h["MILC12_hisq_mass"] < max(bench.HISQ_MASSES)


def test_overlap_workload_is_rbc11():
    t = _golden()["RBC11"]
    o = _golden()["_sec2_3"]
    assert bench.OV_LAT == (t["L"], t["L"], t["L"], t["T"])
    assert bench.OV_M == t["m_overlap"] and bench.OV_RHO == o["rho"]
    assert list(bench.OV_MASSES) == o["overlap_masses"] and bench.OV_MM_TOL == o["overlap_tolerance"]

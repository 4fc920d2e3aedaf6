"""The stored SDF footprint counts match the oracle on the current generator.

The full roofline workload takes over a minute to regenerate, so the
differentiation workload (same generator, 4.1e6 taxels) is recounted here.
"""
import json
import os

import oracle
from paper_2408_06506_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sdf_footprint.json")


def test_stored_footprint_matches_oracle():
    with open(GOLDEN) as f:
        stored = json.load(f)["workloads"]
    sc = wl.make_c5()
    rec = stored["differentiation_1024x2x40x50_128"]
    assert rec["n_taxels"] == sc.n_taxels and rec["n_inst"] == sc.n_inst
    assert oracle.footprint(sc, oracle.state64(sc)) == rec["nodes"]
    # a union is at most every stencil node and at least one node per taxel in the grid box
    c3 = stored["roofline_8192x2x80x100_256"]
    assert c3["n_taxels"] // 8 < c3["nodes"] < 32 * c3["n_taxels"]

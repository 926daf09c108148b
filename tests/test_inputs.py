"""The workloads that stand for the paper's simulations carry the parameters
of its Table I (tests/golden/table1_parameters.txt)."""
import os

import numpy as np

from paper_1501_05630_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_parameters.txt")
NAMES = {"2d": "table1_2d_gauss", "chimera": "table1_chimera_gauss", "3d": "table1_3d_gauss"}


def read_table1():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            top, ns, nsa, b, tmin, tmax, nt, nc = line.split()
            rows[top] = dict(N=[int(x) for x in ns.split(",")], n_sa=int(nsa), b=int(b),
                             t_min=float(tmin), t_max=float(tmax), n_t=int(nt), n_c=int(nc))
    return rows


def test_table1_workloads_match_the_paper():
    rows = read_table1()
    assert set(rows) == set(NAMES)
    for top, row in rows.items():
        spec = inputs.WORKLOADS[NAMES[top]]
        assert [inputs.n_sites(spec["topology"], L) for L in spec["sides"]] == row["N"]
        assert spec["per_side"] == row["n_sa"]
        assert spec["n_instances"] == row["n_sa"] * len(row["N"])
        assert spec["n_sweeps"] == 1 << row["b"]
        assert spec["n_temps"] == row["n_t"] and spec["n_icm"] == row["n_c"]
        assert spec["kind"] == "gauss" and spec["n_replicas"] == 2
        # one instance per size: the temperatures span the table's range and
        # the cluster moves go to the n_c coldest
        for si, L in enumerate(spec["sides"]):
            J, temps, kc, sp = inputs.workload_instance(NAMES[top], si * spec["per_side"])
            assert sp["L"] == L and kc == row["n_c"]
            assert len(temps) == row["n_t"] and np.all(np.diff(temps) > 0)
            assert abs(temps[0] - row["t_min"]) < 1e-12 and abs(temps[-1] - row["t_max"]) < 1e-12
            assert J.shape[0] == (L * L if spec["topology"] == inputs.CHIMERA else row["N"][si])

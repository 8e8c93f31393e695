"""The Gset command line on the GPU: solve a Gset file, write the best
state as a hexadecimal string, and verify it on the host."""
import json

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import gset
from paper_2311_09275_amd import instances as I

pytestmark = pytest.mark.gpu


def test_solve_and_verify(tmp_path, capsys):
    inst = I.torus(20, 14, 9)
    g = tmp_path / "torus.txt"
    gset.write_gset(inst, g)
    hx = tmp_path / "best.txt"
    gset.main(["solve", str(g), "--sweeps", "300", "--replicas", "32", "--beta0", "0.1",
               "--beta1", "3.0", "--seed", "5", "--target", "100", "--hex-out", str(hx)])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    o = O.anneal(inst, 300, 32, 5, kind=O.LINEAR, beta0=0.1, beta1=3.0, want_states=False)
    assert out["best_cut"] == int(o.best_cut.max())
    assert out["ps"] == float(np.mean(o.best_cut >= 100))
    gset.main(["verify", str(g), str(hx)])
    assert int(capsys.readouterr().out.strip()) == out["best_cut"]


def test_solve_with_tempering(tmp_path, capsys):
    inst = I.torus(16, 12, 10)
    g = tmp_path / "torus.txt"
    gset.write_gset(inst, g)
    gset.main(["solve", str(g), "--sweeps", "120", "--temps", "4", "--sets", "4",
               "--swap-every", "5", "--beta0", "0.3", "--beta1", "2.0", "--seed", "6",
               "--cluster-from", "2", "--target", "150"])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    o = O.temper(inst, list(np.geomspace(0.3, 2.0, 4)), 4, 120, 5, 6, cluster_from=2)
    assert out["best_cut"] == int(o.best_cut.max())
    assert out["ps"] == float(np.mean(o.best_cut.reshape(4, 4).max(axis=1) >= 150))

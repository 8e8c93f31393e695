"""The Gset command line on the GPU: solve a Gset file, write the best
state as a hexadecimal string, and verify it on the host."""
import ast

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
    out = ast.literal_eval(capsys.readouterr().out.strip().splitlines()[-1])
    o = O.anneal(inst, 300, 32, 5, kind=O.LINEAR, beta0=0.1, beta1=3.0, want_states=False)
    assert out["best_cut"] == int(o.best_cut.max())
    assert out["ps"] == float(np.mean(o.best_cut >= 100))
    gset.main(["verify", str(g), str(hx)])
    assert int(capsys.readouterr().out.strip()) == out["best_cut"]

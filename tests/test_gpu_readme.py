"""The quick-start example of the README runs as written, and its results are right: the matvec and
the lowest Lanczos eigenvalue against the oracle, the coupling gradient against its closed form."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_readme_quick_start():
    text = open(os.path.join(os.path.dirname(__file__), "..", "README.md")).read()
    code = text.split("```python\n", 1)[1].split("```", 1)[0]
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    from oracle import mf
    from oracle import kron
    from workloads.model import Model
    m = Model(ns["sites"], ns["terms"], np.array([1.0, 1.2, 0.1]))
    x = ns["x"].detach().cpu().numpy()
    assert np.linalg.norm(ns["y"].cpu().numpy() - mf.matvec(m, x)) <= 1e-12 * np.linalg.norm(mf.matvec(m, x))
    e0 = np.linalg.eigvalsh(kron.dense_H(m, m.theta))[0]
    assert abs(ns["out"]["result"].cpu().numpy()[0] - e0) <= 1e-10
    # d/dtheta_p Re <x|H|x> = Re <x|h_p x>
    from oracle import grad as ograd
    _, gt = ograd.adjoint(m, x, x)
    assert np.max(np.abs(ns["theta"].grad.cpu().numpy() - gt)) <= 1e-12 * max(1.0, np.max(np.abs(gt)))

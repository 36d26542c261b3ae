"""Pin of the oracle's hand-written adjoint against central finite
differences of the oracle's own forward run (the forward is pinned
separately).  Objective: drag or torque of the state after n steps from
the inflow Maxwellian; parameters: wall temperature, Knudsen number and the
farfield velocity components."""
import dataclasses

import numpy as np
import pytest

from ccdvm_inputs import Body, small_2d
from oracle import Oracle2D


def objective(cfg, n, obj):
    o = Oracle2D(cfg)
    f, g = o.init()
    f, g, _ = o.run(f, g, n)
    d = o.force(*o.merge(f, g))
    return d[0] if obj == "drag" else d[2]


CASES = [
    ("drag", small_2d(12, 10, 8, kn=0.1, mach=0.5,
                      body=Body("ellipse", (0.47, 0.52, 0), (0.22, 0.12, 0), theta=0.4, t_wall=1.3))),
    ("torque", small_2d(12, 10, 8, kn=0.1, mach=0.5,
                        body=Body("ellipse", (0.47, 0.52, 0), (0.22, 0.12, 0), theta=0.4, t_wall=1.3))),
    ("drag", small_2d(10, 10, 6, kn=0.0, mach=0.8,
                      body=Body("circle", (0.5, 0.52, 0), (0.24, 0.24, 0), t_wall=0.7))),
    ("drag", small_2d(6, 6, 4, kn=0.07, mach=0.4, body=Body("circle", (0.5, 0.52, 0), (0.19, 0.19, 0)))),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_adjoint_matches_central_differences(k):
    obj, cfg = CASES[k]
    n = 6
    J, grad = Oracle2D(cfg).adjoint(n, obj)
    assert J == pytest.approx(objective(cfg, n, obj), rel=1e-13)
    h = 1e-5
    b = cfg.body

    def with_tw(t):
        return cfg.with_(body=dataclasses.replace(b, t_wall=t))

    def with_u(d, du):
        inf = list(cfg.inflow)
        inf[1 + d] += du
        return cfg.with_(inflow=tuple(inf))

    fd = [(objective(with_tw(b.t_wall + h), n, obj) - objective(with_tw(b.t_wall - h), n, obj)) / (2 * h)]
    if cfg.kn > 0:
        fd.append((objective(cfg.with_(kn=cfg.kn * (1 + h)), n, obj)
                   - objective(cfg.with_(kn=cfg.kn * (1 - h)), n, obj)) / (2 * h * cfg.kn))
    else:
        fd.append(0.0)
    for d in (0, 1):
        fd.append((objective(with_u(d, h), n, obj) - objective(with_u(d, -h), n, obj)) / (2 * h))
    scale = max(np.max(np.abs(fd)), 1e-12)
    for a, f in zip(grad, fd):
        # central differences carry O(h^2) truncation and ~1e-16/h rounding
        assert abs(a - f) <= 1e-6 * scale, (grad, fd)

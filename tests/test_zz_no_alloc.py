"""cc_bind_noalloc (the library's static scratch array) against cc_bind (a
caller scratch buffer).  Both run the same kernels on the same buffers, so the
states, the diagnostic rows, the moments and the body state must agree
bitwise.  Two contexts in a row, the second on a smaller input (a moving
body, whose per-step lists also live in the scratch), take the array over in
turn; the first then reports CC_ESTATE until it is bound again."""
import math

import numpy as np
import pytest

from ccdvm_inputs import Body, random_state, small_2d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_04544_amd.solver import Solver  # noqa: F401 (fails loudly if unbuilt)


FIXED = small_2d(72, 40, 16, kn=0.1, mach=0.6)            # several tiles, ragged rows
MOVING = small_2d(40, 32, 8, kn=0.1, mach=0.5, body=Body(
    "ellipse", (0.5, 0.5, 0), (0.15, 0.06, 0), theta=math.pi / 8, motion="free_rotation", inertia=0.002))


def run(cfg, static, nsteps, seed):
    from paper_1503_04544_amd.solver import Solver
    s = Solver(cfg, device="cuda:0", static_scratch=static)
    f0, g0 = random_state(cfg.ncell, cfg.nv, 2, seed=seed)
    s.load_state(torch.from_numpy(f0), torch.from_numpy(g0))
    d = s.step(nsteps, diag=True)
    f, g = s.store_state()
    m = s.moments()
    torch.cuda.synchronize()
    return s, [f.cpu().numpy(), g.cpu().numpy(), d.cpu().numpy(), m.cpu().numpy(), s.body_state()]


def test_noalloc_equals_bind_on_two_calls_in_a_row():
    from paper_1503_04544_amd._capi import CCError
    print("noalloc: fixed cylinder 72x40, 16^2 velocities, 8 steps", flush=True)
    ref, want = run(FIXED, False, 8, 31)
    first, got = run(FIXED, True, 8, 31)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    ref.close()
    print("noalloc: moving ellipse 40x32, 8^2 velocities, 6 steps", flush=True)
    ref2, want2 = run(MOVING, False, 6, 32)
    second, got2 = run(MOVING, True, 6, 32)
    for a, b in zip(got2, want2):
        assert np.array_equal(a, b)
    # the second context took the array over: the first must be bound again
    with pytest.raises(CCError) as e:
        first.step(1)
    assert e.value.status == -6
    ref2.close()
    second.close()
    first.close()

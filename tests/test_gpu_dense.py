"""The folded dense transforms of A_p^{-1} (Section 3.3's sine / cosine
transforms as two half-size matrix products, xform_dense.hip) against the
FP64 oracle for every line length L = 1 .. 150 and a few long ones, odd and
even (with and without a middle node), on x lines and y columns, in both
bases; H6_DENSE_TRANSFORMS keeps the FFT paths out."""
import numpy as np
import pytest

import oracle
from paper_1212_1397_amd.workloads import random_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("prec,bound", [("fp64", 1e-12), ("mixed", 5e-5)])
def test_dense_every_line_length(monkeypatch, axis, prec, bound):
    from paper_1212_1397_amd import helmholtz6 as h6
    monkeypatch.setenv("H6_DENSE_TRANSFORMS", "1")
    worst = 0.0
    ns = list(range(1, 149)) + [191, 254, 255, 256, 300]
    for n_line in ns:
        for basis in ("D", "N"):
            n = [2, 2, 2]
            n[axis] = n_line
            bc = ["D", "D", "D", "D", "D", "D"]
            bc[2 * axis] = bc[2 * axis + 1] = basis
            bc = "".join(bc)
            prob = oracle.Problem(tuple(n), 1.0 / (max(n) + 1), 3.0 + 0.2j, tuple(bc))
            x = random_field(prob.shape, seed=n_line)
            plan = h6.Plan(prob.n, prob.h, prob.k, bc, precision=prec)
            z = plan.apply_Pinv(torch.from_numpy(x).cuda()).cpu().numpy()
            plan.close()
            e = relerr(z, oracle.apply_Pinv(prob, x))
            worst = max(worst, e)
            assert e <= bound, (axis, n_line, basis, e)
    print(f"axis {axis} {prec}: worst relative error {worst:.1e}", flush=True)

"""Pin of the oracle's three-dimensional Robin transmission rows (Section 5.2.1:
the condition of eq. contRob, its forward-difference form eq. discRob and the
extension row eq. robfo, with the subsurface closest point of eq. locCP and
the conormal of eq. naConorm) by the condition they discretise.

For a boundary node b of subdomain j with effective boundary point
y = CP_{S_j}(x_b) and conormal q (computed here independently, by brute force
over the closest points of the final overlap layer), the surface function
    g_b(p) = exp(-alpha q.(p - y))
satisfies the Robin condition dg/dq + alpha g = 0 at y exactly. Sampled the
way the closest point method represents surface functions (u_i = g_b(CP(x_i))
for every local unknown, including u_b itself), the oracle's B row of A_j
(eq. localOP), scaled by h^2/6, must vanish to second order in h for fixed
alpha: the row interpolates g_b at y to fourth order and the forward
difference of eq. discRob is exact to first order in s_b = d.q, whose
remainder alpha^2 s_b^2 is O(h^2), as is the c h^2/6 term of the row.

A function that violates the condition (dg/dq = +alpha g) leaves a first-order
defect 2 alpha s_b, and so do plausible mistakes in the row, planted here in
the oracle's decomposition: the sign of the Robin term (1/(1 - alpha s)), the
division dropped (plain extension), and the conormal taken without removing
the normal component of d (s = |d|).
"""

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
from oracle import schwarz

ALPHA = 1.0
C = 1.0
# (h, RCB parts): about 2-5 thousand local unknowns each
GRIDS = [(0.1, 8), (0.05, 16), (0.025, 64)]


def _robin_defects(band, dec, j, sign):
    """|h^2/6 (A_j g_b)_b| for every B node of subdomain j with s_b > 0."""
    surf = ci.Sphere()
    sd = dec.subs[j]
    A = schwarz.local_matrix(band, dec, j, C)
    m = len(sd.sigma)
    cp_unk = band.cp[np.concatenate([sd.sigma, sd.bnd])]
    cf = band.cp[sd.final]
    h2 = band.h * band.h
    out = []
    for ib, node in enumerate(sd.bnd):
        xb = band.xyz[node]
        y = cf[np.argmin(((xb - cf) ** 2).sum(axis=1))]  # eq. locCP, brute force
        _, nrm = surf.cp(y[None, :])
        n = nrm[0]
        d = xb - y
        t = d - (d @ n) * n                               # eq. naConorm before normalising
        s = np.linalg.norm(t)
        if s == 0.0:
            continue
        q = t / s
        row = A[m + ib]
        nz = np.flatnonzero(row)
        g = np.exp(sign * ALPHA * ((cp_unk[nz] - y) @ q))
        out.append(abs(row[nz] @ g) / (6.0 / h2))
    return np.array(out)


def _mutate(dec, j, band, how):
    sd = dec.subs[j]
    if how == "sign":
        sd.s = -sd.s
    elif how == "no_division":
        sd.s = np.zeros_like(sd.s)
    elif how == "no_projection":
        sd.s = np.linalg.norm(band.xyz[sd.bnd] - band.cp[sd.xstar], axis=1)


@pytest.fixture(scope="module")
def defects():
    """Largest defect per grid for the true row with g satisfying the
    condition, g violating it, and each planted mistake."""
    cases = [("row", -1.0, None), ("violating_g", 1.0, None), ("sign", -1.0, "sign"),
             ("no_division", -1.0, "no_division"), ("no_projection", -1.0, "no_projection")]
    res = {name: [] for name, _, _ in cases}
    for h, n_sub in GRIDS:
        band = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
        part = oracle.rcb_partition(band, n_sub)
        for name, sign, how in cases:
            dec = schwarz.decompose(band, part, 2, "ORAS", alpha=ALPHA, only={0})
            if how:
                _mutate(dec, 0, band, how)
            dd = _robin_defects(band, dec, 0, sign)
            assert len(dd) > 500
            res[name].append(dd.max())
    return res


def _slope(vals):
    hs = np.array([h for h, _ in GRIDS])
    return float(np.polyfit(np.log(hs), np.log(np.array(vals)), 1)[0])


def test_robin_row_is_second_order_consistent(defects):
    assert _slope(defects["row"]) >= 1.7, defects["row"]
    assert defects["row"][-1] < 0.01


@pytest.mark.parametrize("name", ["violating_g", "sign", "no_division", "no_projection"])
def test_wrong_condition_or_planted_mistake_leaves_first_order_defect(defects, name):
    assert _slope(defects[name]) <= 1.3, defects[name]
    assert defects[name][-1] > 5 * defects["row"][-1]

"""Oracle results at single nodes of grids too large for the whole-field
oracle: the oracle steps a small periodic patch cut out of the input fields
around the node.

One step of the method at a node reads the streamed populations of the node
(one node away) and the anomaly of its neighbours, whose moments pull from
one node further: two nodes in all.  The moments after a step are those of
the populations streamed into the node, which carry no collision of that
step.  So the moments at a node after s steps depend on the initial state
within 2 (s - 1) + 1 nodes of it: 3 for two steps.  A patch of radius 4
(9^3 nodes) stepped twice with periodic wrap therefore gives the whole grid's
moments at its centre; tests/test_oracle_patch.py checks this against the
whole-field oracle.  Nothing here comes from the GPU library.
"""
import numpy as np

import oracle


def patch(a, x, y, z, n, r=4):
    """The (2r+1)^3 block of a periodic (n, n, n) array (z, y, x order)
    centred on (x, y, z)."""
    ix = (x + np.arange(-r, r + 1)) % n
    iy = (y + np.arange(-r, r + 1)) % n
    iz = (z + np.arange(-r, r + 1)) % n
    return a[np.ix_(iz, iy, ix)]


def two_step_moments(fields, node, n, sim_kw, rest=None, band=0.0, r=4):
    """rho, u, T at node (flat index into an n^3 periodic grid) after two
    oracle steps from the equilibria of fields, computed on a radius-r patch.
    rest: reference populations (f_ref, g_ref) of the FP32 storage model, or
    None.  Returns the moments, the patch's velocities after step 1 within
    one node of the centre (those that set the upwind sides of the step-1
    collisions the centre's moments depend on) and, when any of them is
    within band of zero, the moments with those sides reversed (else None)."""
    rho, u, T = fields
    z, rem = divmod(int(node), n * n)
    y, x = divmod(rem, n)
    pr = patch(rho, x, y, z, n, r)
    pu = np.stack([patch(u[a], x, y, z, n, r) for a in range(3)])
    pT = patch(T, x, y, z, n, r)
    w = 2 * r + 1

    def run(b):
        s = oracle.Sim(3, (w, w, w), **sim_kw)
        if rest is not None:
            s.set_fp32_storage(*rest)
        if b:
            s.set_upwind_band(b)
        s.init(pr, pu, pT)
        s.step(1)
        u1 = s.moments()[1][:, r - 1:r + 2, r - 1:r + 2, r - 1:r + 2].copy()
        s.step(1)
        m = s.moments()
        return (float(m[0][r, r, r]), m[1][:, r, r, r].copy(), float(m[2][r, r, r])), u1

    plain, u1 = run(0.0)
    alt = run(band)[0] if band > 0 and (np.abs(u1) <= band).any() else None
    return plain, u1, alt

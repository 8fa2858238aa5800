"""Weight-window centre tables for tests, built from an analog flux tally of
the oracle: w_c(cell) = phi(cell) / phi(source cell), the forward-flux
window normalised to the source weight (0 where the flux is 0 = no window).
The table is test input, computed with NumPy from the oracle's estimate."""
import numpy as np

import oracle


def flux_table(prob, N=20000, seed=99, floor=1e-6):
    res = oracle.run(prob, N, seed)
    e = oracle.estimates(prob, res)
    phi = e["mean"]                                  # [K, G, nz, ny, nx]
    src = prob["source"]
    mesh = prob["ww_mesh"]
    idx = []
    for a in (2, 1, 0):
        m = mesh[a]
        c = 0.5 * (src["lo"][a] + src["hi"][a])
        idx.append(int(np.clip(np.searchsorted(m, c, side="right") - 1, 0, m.size - 2)) if m.size else 0)
    ref = phi[0, 0, idx[0], idx[1], idx[2]]
    w = phi / ref
    w[w < floor] = 0.0
    return np.ascontiguousarray(w)

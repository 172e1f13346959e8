"""Shared helpers of the GPU parity tests: problem conversion, order-map
comparison with the decision bands, and relative state errors."""
import numpy as np

import oracle

THETA_BAND = 1e-12      # |psi^p - theta| within this: decision may flip
PSI1_BAND = 1e-12       # |u_{i+1,c} - u_{i,c}| <= band * max|u_c|: superbee may jump


def both_problems(dim, nvar, nx, flux, P, bc, dx, ny=1, dy=1.0, gamma=1.4, ax=1.0, ay=1.0, flags=0):
    import paper_2007_01416_amd as acat
    fid = {"advection": oracle.FLUX_ADVECTION, "burgers": oracle.FLUX_BURGERS, "euler": oracle.FLUX_EULER}[flux]
    bid = {"periodic": oracle.BC_PERIODIC, "transmissive": oracle.BC_TRANSMISSIVE}[bc]
    po = oracle.Problem(dim=dim, nvar=nvar, nx=nx, ny=ny, flux=fid, P=P, bc=bid, gamma=gamma, ax=ax, ay=ay,
                        dx=dx, dy=dy, flags=flags)
    pg = acat.Problem(dim=dim, nvar=nvar, nx=nx, ny=ny, flux=flux, P=P, bc=bc, gamma=gamma, ax=ax, ay=ay, dx=dx,
                      dy=dy, flags=flags)
    return po, pg


def from_workload(w, **over):
    kw = dict(dim=w["dim"], nvar=w["nvar"], nx=w["u"].shape[-1], flux=w["flux"], P=w["P"], bc=w["bc"], dx=w["dx"],
              gamma=w.get("gamma", 1.4))
    if w["dim"] == 2:
        kw.update(ny=w["u"].shape[1], dy=w["dy"])
    kw.update(over)
    return both_problems(**kw)


def line_values(u, dim, d, k_entry, row, bc, G):
    """Values of every component along direction d around interface entry
    k_entry (1D: row ignored), offsets -G+1..G, as the oracle indexes them."""
    nv = u.shape[0]
    off = 0 if bc == oracle.BC_PERIODIC else -1
    i = k_entry + off
    out = np.zeros((nv, 2 * G))
    for a in range(2 * G):
        j = i - G + 1 + a
        if dim == 1:
            n = u.shape[1]
            jj = j % n if bc == oracle.BC_PERIODIC else min(max(j, 0), n - 1)
            out[:, a] = u[:, jj]
        else:
            n = u.shape[2] if d == 0 else u.shape[1]
            jj = j % n if bc == oracle.BC_PERIODIC else min(max(j, 0), n - 1)
            out[:, a] = u[:, row, jj] if d == 0 else u[:, jj, row]
    return out


def in_band(vals, P, theta=0.5, eps=1e-12):
    """True if the decision at this interface is within a decision band."""
    G = max(P, 2)
    for p in range(2, P + 1):
        psi = min(oracle.indicator(vals[c, G - p:G + p], p, eps) for c in range(vals.shape[0]))
        if abs(psi - theta) <= THETA_BAND:
            return True
    for c in range(vals.shape[0]):
        dl = vals[c, G] - vals[c, G - 1]
        if abs(dl) <= PSI1_BAND * max(np.abs(vals[c]).max(), 1e-300):
            return True
    return False


def order_mismatches(u, ord_o, ord_g, dim, d, bc, P):
    """(#mismatches outside the bands, #mismatches inside the bands)."""
    bad = np.argwhere(np.asarray(ord_o) != np.asarray(ord_g))
    outside = inside = 0
    G = max(P, 2)
    for idx in bad:
        if dim == 1:
            vals = line_values(u, 1, 0, idx[0], 0, bc, G)
        elif d == 0:        # x-interfaces [row][k]
            vals = line_values(u, 2, 0, idx[1], idx[0], bc, G)
        else:               # y-interfaces [k][col]
            vals = line_values(u, 2, 1, idx[0], idx[1], bc, G)
        if in_band(vals, P):
            inside += 1
        else:
            outside += 1
    return outside, inside


def rel_err(a, b):
    """max over components of max|a_c - b_c| / max|b_c|."""
    a = np.asarray(a); b = np.asarray(b)
    errs = []
    for c in range(a.shape[0]):
        scale = max(np.abs(b[c]).max(), 1e-300)
        errs.append(np.abs(a[c] - b[c]).max() / scale)
    return max(errs)

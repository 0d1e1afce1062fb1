"""Error measures for comparing the HIP path with the oracle.

Cell averages: per component, max over cells of |gpu - ref| divided by a scale of that component:
max |h| for thicknesses, max h sqrt(G h) (momentum of a wave-speed flow) for momenta, so that
momenta near zero (rest states) are measured against the flow's natural size.  Gradients: the same
scale per component, or the largest reference gradient if that is bigger.
"""
import numpy as np

TOL_FP64 = 1e-12  # parity bound for the FP64 path, per step


def scales(Wr, G=9.81):
    s = np.zeros(6)
    for o in (0, 3):
        h = np.abs(Wr[o])
        s[o] = h.max()
        mom = (h * np.sqrt(G * h)).max()
        s[o + 1] = s[o + 2] = mom
    return s


def state_err(W, Wr, G=9.81):
    s = scales(Wr, G)
    return np.array([np.abs(W[v] - Wr[v]).max() / s[v] for v in range(6)])


def grad_err(gW, gWr, Wr, G=9.81):
    s = scales(Wr, G)
    out = np.zeros(6)
    for v in range(6):
        sc = max(s[v], np.abs(gWr[v]).max())
        out[v] = np.abs(gW[v] - gWr[v]).max() / sc
    return out

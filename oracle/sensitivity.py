"""Compliance sensitivities, eq. (6)-(7) (oracle).  Test infrastructure only.

Block RL.2/RL.3 of both codes: dsK = -p (E0 - Emin) xphys^(p-1) on the active
set (0 on passive elements; 0^0 = 1 when p = 1), element energies
ce_e = u_e^T Ke u_e with u_e = u[C[e,:]], dc = dsK . ce, compliance c = f^T u.
"""
import numpy as np


def element_energy(u, cmat, ke_full):
    ue = u[cmat]                       # m x d
    return np.einsum("ei,ij,ej->e", ue, ke_full, ue)


def dsk(xphys, act, penal, E0, Emin):
    out = np.zeros_like(xphys)
    out[act] = -penal * (E0 - Emin) * np.power(xphys[act], penal - 1.0)
    return out


def sensitivity(xphys, u, cmat, ke_full, act, penal, E0, Emin):
    """Returns dc (raw, eq. (7)) and the element energies."""
    ce = element_energy(u, cmat, ke_full)
    return dsk(xphys, act, penal, E0, Emin) * ce, ce


def compliance(f, u):
    return float(f @ u)

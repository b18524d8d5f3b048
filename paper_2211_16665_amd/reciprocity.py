"""Source-receiver reciprocity swap (the marine example of Section 4 switches
sources and receivers for efficiency: 810 source positions, 25 receivers).

For electric dipoles the discrete Green's function is symmetric: the field
component i at r of a unit j-dipole at s equals the field component j at s of
a unit i-dipole at r.  It holds exactly for the stepped system here, because
injection spreads a dipole with the trilinear weights divided by the dual
volume and recording interpolates with the same weights, and under the dual
volumes the discrete curl pair is symmetric.  So the data of Ns sources at
Nr receivers (components c) come from Nr * ncomp runs with a unit c-dipole
at each receiver, recording the three E components at the source positions
and projecting them on each source's moment:

    d[s][r][ci][k] = sum_j p_s[j] E_swap[r * ncomp + ci][s][j][k].

The map is linear, so the misfit and its gradient with respect to ln rho are
those of the original survey (the adjoint of the swapped runs receives the
transposed residual, which torch.autograd forms by itself when the map is
applied to FictitiousForward's output).  This module only moves indices;
every field still comes from the library.  Magnetic data would need magnetic
sources in the swapped runs and are refused.
"""
from __future__ import annotations

import numpy as np


def swap_workload(w):
    """The reciprocal survey of workload ``w`` (electric sources and electric
    receiver components): one source per (receiver, component) with a unit
    moment along that component, receivers at the original source positions
    recording E_x, E_y, E_z."""
    comps = tuple(int(c) for c in w.rec_comp)
    if any(c > 2 for c in comps):
        raise ValueError("the reciprocity swap covers electric receiver components only")
    rec = np.asarray(w.rec_pos, dtype=np.float64)
    pos = np.repeat(rec, len(comps), axis=0)
    mom = np.zeros((len(pos), 3))
    for r in range(len(rec)):
        for ci, c in enumerate(comps):
            mom[r * len(comps) + ci, c] = 1.0
    return w.replace(src_pos=pos, src_mom=mom,
                     rec_pos=np.asarray(w.src_pos, dtype=np.float64).copy(), rec_comp=(0, 1, 2))


def fields_to_data(E_swap, src_mom, ncomp):
    """Data of the original survey [ns][nr][ncomp][nf] from the swapped runs'
    output E_swap [nr * ncomp][ns][3][nf] (numpy array or torch tensor;
    torch keeps the autograd graph)."""
    p = np.asarray(src_mom, dtype=np.float64)
    ns = p.shape[0]
    nsw, ns2, three, nf = E_swap.shape
    if ns2 != ns or three != 3 or nsw % ncomp:
        raise ValueError("E_swap does not match the swapped survey")
    nr = nsw // ncomp
    if isinstance(E_swap, np.ndarray):
        E = E_swap.reshape(nr, ncomp, ns, 3, nf)
        return np.einsum("sj,rcsjk->srck", p, E)
    import torch
    E = E_swap.reshape(nr, ncomp, ns, 3, nf)
    pt = torch.as_tensor(p, dtype=E.dtype, device=E.device)
    # sum over j written out (no batched products on transposed views)
    out = sum(pt[:, j].reshape(1, 1, ns, 1) * E[:, :, :, j, :] for j in range(3))
    return out.permute(2, 0, 1, 3).contiguous()


def residual_to_swapped(resid, src_mom, ncomp):
    """The transpose of fields_to_data: a weighted residual of the original
    survey [ns][nr][ncomp][nf] as the residual of the swapped runs
    [nr * ncomp][ns][3][nf] (for fwd_adjoint on the swapped plan)."""
    p = np.asarray(src_mom, dtype=np.float64)
    R = np.asarray(resid)
    ns, nr, nc, nf = R.shape
    if nc != ncomp or p.shape[0] != ns:
        raise ValueError("residual does not match the survey")
    out = np.einsum("sj,srck->rcsjk", p, R)
    return out.reshape(nr * ncomp, ns, 3, nf)

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
every field still comes from the library.

Magnetic data and magnetic sources follow from Lorentz reciprocity of eq.
freq (curl E - i w mu H = M, curl H - sigma E = J): for two source
distributions, the integral of E_2 . J_1 + H_2 . M_1 equals that of
E_1 . J_2 + H_1 . M_2.  So a component of H at r (from an electric dipole at
s) is the matching E component at s from a unit magnetic dipole at r; E at r
from a magnetic dipole at s is H at s from an electric dipole at r; and H-H
pairs are symmetric like E-E pairs.  The swapped runs therefore use electric
unit sources for the electric receiver components and magnetic ones for the
magnetic components (two plans when both are recorded), and record E at the
source positions when the original sources are electric, H when they are
magnetic.  The stepped system keeps these identities exactly (the H node
volumes make the Faraday and Ampere rows a symmetric pair).
"""
from __future__ import annotations

import numpy as np


def swap_workloads(w):
    """The reciprocal survey of workload ``w`` as a list of (workload,
    component positions): one workload per kind of receiver component
    (electric components 0-2, magnetic 3-5; only kinds ``w`` records), each
    with one unit dipole per (receiver, component) of that kind -- electric
    for E components, magnetic for H components, along the component's axis
    -- and receivers at the original source positions recording the three E
    components (electric original sources) or the three H components
    (magnetic ones).  The positions index w.rec_comp."""
    comps = tuple(int(c) for c in w.rec_comp)
    rec = np.asarray(w.rec_pos, dtype=np.float64)
    rec_comp = (0, 1, 2) if getattr(w, "src_kind", 0) == 0 else (3, 4, 5)
    out = []
    for kind in (0, 1):
        cis = [ci for ci, c in enumerate(comps) if (c >= 3) == (kind == 1)]
        if not cis:
            continue
        pos = np.repeat(rec, len(cis), axis=0)
        mom = np.zeros((len(pos), 3))
        for r in range(len(rec)):
            for g, ci in enumerate(cis):
                mom[r * len(cis) + g, comps[ci] % 3] = 1.0
        out.append((w.replace(src_pos=pos, src_mom=mom, src_kind=kind,
                              rec_pos=np.asarray(w.src_pos, dtype=np.float64).copy(),
                              rec_comp=rec_comp), cis))
    return out


def swap_workload(w):
    """The reciprocal survey of a workload whose receiver components are all
    of one kind (all electric or all magnetic): swap_workloads' one
    workload."""
    parts = swap_workloads(w)
    if len(parts) != 1:
        raise ValueError("electric and magnetic receiver components: use swap_workloads")
    return parts[0][0]


def data_from_swaps(parts, src_mom, ncomp):
    """Data of the original survey [ns][nr][ncomp][nf] from the outputs of
    swap_workloads' runs: ``parts`` lists (E_swap, component positions) with
    E_swap [nr * len(positions)][ns][3][nf] (numpy or torch)."""
    outs = [(fields_to_data(E, src_mom, len(cis)), cis) for E, cis in parts]
    d0 = outs[0][0]
    if isinstance(d0, np.ndarray):
        data = np.zeros(d0.shape[:2] + (ncomp,) + d0.shape[3:], dtype=d0.dtype)
        for d, cis in outs:
            data[:, :, cis] = d
        return data
    import torch
    cols = [None] * ncomp
    for d, cis in outs:
        for g, ci in enumerate(cis):
            cols[ci] = d[:, :, g]
    return torch.stack(cols, dim=2)


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

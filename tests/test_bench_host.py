"""Host logic of bench.py: the one-GPU contract and the algorithmic-byte model
of the roofline (counts of updated edges, H nodes and CPML memory variables
checked against explicit loops over the lattices)."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _in_int(i, n, npml):        # integer node inside a layer (interior nodes 1..n-1)
    return npml > 0 and (i < npml or i > n - npml)


def _in_half(i, n, npml):       # half node inside a layer (0..n-1)
    return npml > 0 and (i < npml or i >= n - npml)


@pytest.mark.parametrize("nx,ny,nz,npml", [(12, 10, 9, 3), (9, 11, 8, 0), (14, 12, 13, 4)])
def test_e_update_byte_model(nx, ny, nz, npml):
    tsize, accsize, kb, nf = 4, 16, 8, 3
    edges = psi = 0
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                if i < nx and 1 <= j < ny and 1 <= k < nz:          # E_x: d/dy, d/dz
                    edges += 1
                    psi += _in_int(j, ny, npml) + _in_int(k, nz, npml)
                if 1 <= i < nx and j < ny and 1 <= k < nz:          # E_y: d/dz, d/dx
                    edges += 1
                    psi += _in_int(k, nz, npml) + _in_int(i, nx, npml)
                if 1 <= i < nx and 1 <= j < ny and k < nz:          # E_z: d/dx, d/dy
                    edges += 1
                    psi += _in_int(i, nx, npml) + _in_int(j, ny, npml)
    b, e = bench.algorithmic_bytes_e(nx, ny, nz, npml, tsize, kb)
    assert e == edges
    assert b == int(edges * (4 * tsize + (kb - 1) * tsize / kb) + psi * 2 * tsize)
    b0, _ = bench.algorithmic_bytes_e(nx, ny, nz, npml, tsize, kb, hist=False)
    assert b0 == edges * 4 * tsize + psi * 2 * tsize
    # block transform: kb samples and the accumulators' read + write per edge
    assert bench.algorithmic_bytes_transform(edges, nf, tsize, accsize, kb) == \
        edges * (kb * tsize + 2 * nf * accsize)
    assert bench.algorithmic_bytes_transform(edges, nf, tsize, accsize, kb, adjoint=True) == \
        edges * (kb * tsize + nf * accsize + 16)
    # the first block of a run only writes its accumulators: over a run of
    # 2 blocks the launches average 1.5 accumulator passes
    assert bench.algorithmic_bytes_transform(edges, nf, tsize, accsize, kb, blocks=2) == \
        int(edges * (kb * tsize + 1.5 * nf * accsize))
    assert bench.algorithmic_bytes_transform(edges, nf, tsize, accsize, kb, blocks=1) == \
        edges * (kb * tsize + nf * accsize)


@pytest.mark.parametrize("nx,ny,nz,npml", [(12, 10, 9, 3), (9, 11, 8, 0)])
def test_h_update_byte_model(nx, ny, nz, npml):
    tsize = 4
    hnodes = enodes = psi = 0
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                if j < ny and k < nz:                               # H_x: d/dy, d/dz
                    hnodes += 1
                    psi += _in_half(j, ny, npml) + _in_half(k, nz, npml)
                if i < nx and k < nz:                               # H_y: d/dz, d/dx
                    hnodes += 1
                    psi += _in_half(k, nz, npml) + _in_half(i, nx, npml)
                if i < nx and j < ny:                               # H_z: d/dx, d/dy
                    hnodes += 1
                    psi += _in_half(i, nx, npml) + _in_half(j, ny, npml)
                enodes += (i < nx) + (j < ny) + (k < nz)            # every E node, read once
    assert bench.algorithmic_bytes_h(nx, ny, nz, npml, tsize) == \
        hnodes * 2 * tsize + enodes * tsize + psi * 2 * tsize

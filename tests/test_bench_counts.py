"""The per-row counts behind the bench line's roofline (CPU only): the FLOP
count of the ring-form row (Lemma, eq. correctionterm3D, opposite directions
sharing the reference stencil) follows from the edge patches of the refined
lattice, and the algorithmic bytes and peaks from their definitions."""
import collections

import numpy as np

import bench
from oracle.mesh import reference_refinement


def _edge_patch_sizes(level=3):
    """Number of elements around each of the 14 edges at an interior node of
    the Bey-refined reference macro."""
    ijk, tets = reference_refinement(level)
    n = 1 << level
    node = int(np.nonzero((ijk == [2, 2, 2]).all(1))[0][0])
    assert ijk[node].min() >= 1 and ijk[node].sum() <= n - 1      # macro-interior
    around = tets[(tets == node).any(1)]
    count = collections.Counter()
    for t in around:
        for v in t:
            if v != node:
                count[int(v)] += 1
    return around.shape[0], sorted(count.values())


def test_edge_patches():
    n_el, sizes = _edge_patch_sizes()
    assert n_el == 24 and len(sizes) == 14
    assert sizes == [4] * 6 + [6] * 8


def test_flop_count_of_the_ring_form_row():
    """Per direction with m elements around its edge (m ring nodes, m/2
    reflected pairs): 3 differences of x, m - 1 additions for the ring sum,
    1 for the end points, m/2 differences of k; 1 multiplication (ring weight);
    fused multiply-adds: 1 (k-hat), 3 (k-hat times the difference of x),
    3 m/2 (correction axis), 6 (cross product).  Per pair of opposite
    directions one symmetric 3x3 product, 9 fused multiply-adds.  A fused
    multiply-add counts 2."""
    _, sizes = _edge_patch_sizes()
    adds = muls = fmas = 0
    for m in sizes:
        adds += 3 + (m - 1) + 1 + m // 2
        muls += 1
        fmas += 1 + 3 + 3 * (m // 2) + 6
    fmas += 9 * (len(sizes) // 2)
    assert (adds, muls, fmas) == (150, 14, 311)
    assert 2 * fmas + adds + muls == bench.FLOP_PER_INTERIOR_NODE


def test_bytes_and_peaks():
    # x (3 components) and k read, y (3 components) written, per precision
    assert bench.BYTES_PER_INTERIOR_NODE == {"f64": (3 + 1 + 3) * 8.0, "f32": (3 + 1 + 3) * 4.0}
    # 256 compute units x 2.4 GHz x 64 FP64 FMA lanes x 2 FLOP
    assert abs(256 * 2.4e9 * 64 * 2 / 1e12 - bench.FP64_VECTOR_PEAK_TFLOPS) < 0.05
    assert bench.HBM_PEAK_GBS == 8000.0

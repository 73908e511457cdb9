"""Pins for the oracle's periodic Voronoi tessellation (Sec. 3 of the paper).

The tessellation has a plain definition (each cell is the set of points
closer to its generator than to any other generator image), so the oracle is
pinned by closed forms (the body-centred cubic cell), brute force against the
distance-ordered path with its early stop, and exact geometric identities.
"""
import math

import numpy as np
import pytest

import workloads as W


def directed_faces(m):
    own = m.face_owner()
    return set(zip(own.tolist(), m.j.tolist(), m.code.tolist()))


def test_bcc_closed_form(orc):
    # Body-centred cubic lattice with cube side a: every cell is a truncated
    # octahedron of volume a^3/2 with 6 squares of area a^2/8 (neighbours at
    # distance a) and 8 regular hexagons of area 3 sqrt(3) a^2/16 (neighbours
    # at sqrt(3) a/2); the centroid is the generator.
    m_side = 4
    a = 1.0 / m_side
    pos = W.bcc_lattice(m_side)
    for method in ("brute", "grid"):
        m = orc.tessellate(pos, (1, 1, 1), method=method)
        assert m.status == 0
        np.testing.assert_allclose(m.V, a ** 3 / 2, rtol=1e-13)
        np.testing.assert_allclose(m.c, pos, atol=1e-15)
        nf = np.diff(m.off)
        assert np.all(nf == 14)
        own = m.face_owner()
        dr = m.pos[m.j] - m.pos[own]
        dr -= np.round(dr)          # nearest image in the unit box
        dist = np.linalg.norm(dr, axis=1)
        sq = np.isclose(dist, a, rtol=1e-12)
        hx = np.isclose(dist, math.sqrt(3) * a / 2, rtol=1e-12)
        assert sq.sum() == 6 * m.n and hx.sum() == 8 * m.n
        np.testing.assert_allclose(m.A[sq], a * a / 8, rtol=1e-13)
        np.testing.assert_allclose(m.A[hx], 3 * math.sqrt(3) * a * a / 16, rtol=1e-13)
        # Face centroids of a centrally symmetric cell lie at the bisector feet.
        mid = m.pos[own] + 0.5 * dr
        np.testing.assert_allclose(m.f, mid, atol=1e-15)


CASES = [
    ("lattice", 2), ("lattice", 3), ("lattice", 4), ("lattice", 5), ("lattice", 8),
    ("poisson", 8), ("poisson", 64), ("poisson", 512),
]


@pytest.mark.parametrize("kind,size", CASES)
def test_brute_force_equals_grid(orc, kind, size):
    if kind == "lattice":
        pos = W.jittered_lattice((size,) * 3, (1, 1, 1), seed=10 + size)
    else:
        pos = W.poisson_points(size, (1, 1, 1), seed=20 + size)
    mb = orc.tessellate(pos, (1, 1, 1), method="brute")
    mg = orc.tessellate(pos, (1, 1, 1), method="grid", certificate=True)
    assert mb.status == 0 and mg.status == 0
    assert mg.delta_min > 1e-12, "input is not certified non-degenerate"
    np.testing.assert_array_equal(mb.off, mg.off)
    np.testing.assert_array_equal(mb.j, mg.j)
    np.testing.assert_array_equal(mb.code, mg.code)
    np.testing.assert_allclose(mg.V, mb.V, rtol=1e-13)
    np.testing.assert_allclose(mg.A, mb.A, rtol=1e-11, atol=1e-15 * mb.V.mean() ** (2 / 3))
    np.testing.assert_allclose(mg.c, mb.c, atol=1e-13)
    np.testing.assert_allclose(mg.f, mb.f, atol=1e-12)


def test_exhaustive_brute_force_matches_skip(orc):
    # The farthest-vertex skip used by brute force is exact; without it the
    # result is the same.
    pos = W.poisson_points(27, (1, 1, 1), seed=5)
    a = orc.tessellate(pos, (1, 1, 1), method="brute", exhaustive=True)
    b = orc.tessellate(pos, (1, 1, 1), method="brute", exhaustive=False)
    np.testing.assert_array_equal(a.j, b.j)
    np.testing.assert_array_equal(a.code, b.code)
    np.testing.assert_allclose(a.V, b.V, rtol=1e-13)


def _invariants(m, box, rtol_face=1e-9):
    n = m.n
    L = np.asarray(box)
    # Cells tile the box.
    assert abs(m.V.sum() / np.prod(L) - 1) < 1e-12
    # Independent tetrahedral volumes agree with the pyramid volumes.
    np.testing.assert_allclose(m.vtet, m.V, rtol=1e-12)
    own = m.face_owner()
    # Symmetric topology and A_ij = A_ji.
    key = {(i, j, c): t for t, (i, j, c) in enumerate(zip(own.tolist(), m.j.tolist(), m.code.tolist()))}
    for (i, j, c), t in key.items():
        t2 = key.get((j, i, 26 - c))
        assert t2 is not None, f"face ({i},{j},{c}) has no partner"
        assert abs(m.A[t] - m.A[t2]) <= rtol_face * m.A[t] + 1e-15 * m.V.mean() ** (2 / 3)
    # Closed surfaces: sum_j A n = 0 and sum_j A (f - r_i) n^T = V I.
    k = np.stack([m.code % 3 - 1, (m.code // 3) % 3 - 1, m.code // 9 - 1], axis=1)
    d = m.pos[m.j] + k * L - m.pos[own]
    nh = d / np.linalg.norm(d, axis=1, keepdims=True)
    S = np.zeros((n, 3))
    np.add.at(S, own, m.A[:, None] * nh)
    scale = m.V.mean() ** (2 / 3)
    assert np.abs(S).max() < 1e-13 * scale
    T = np.zeros((n, 3, 3))
    np.add.at(T, own, m.A[:, None, None] * (m.f - m.pos[own])[:, :, None] * nh[:, None, :])
    err = T - m.V[:, None, None] * np.eye(3)[None]
    assert np.abs(err).max() < 1e-13 * m.V.mean()


@pytest.mark.parametrize("shape,box", [((8, 8, 8), (1, 1, 1)), ((16, 4, 4), (4, 1, 1)),
                                        ((6, 5, 7), (1.2, 1.0, 1.4))])
def test_geometric_invariants_lattice(orc, shape, box):
    pos = W.jittered_lattice(shape, box, seed=7)
    m = orc.tessellate(pos, box, method="grid")
    _invariants(m, box)


def test_geometric_invariants_poisson(orc):
    pos = W.poisson_points(2000, (1, 1, 1), seed=8)
    m = orc.tessellate(pos, (1, 1, 1), method="grid")
    _invariants(m, (1, 1, 1))


def test_single_point_is_the_box(orc):
    # One generator: its cell is the whole periodic box, bounded by the
    # bisectors of its own six axis images.
    pos = np.array([[0.3, 0.6, 0.1]])
    for method in ("brute", "grid"):
        m = orc.tessellate(pos, (2, 1, 0.5), method=method)
        assert abs(m.V[0] - 1.0) < 1e-15
        assert sorted(m.code.tolist()) == [4, 10, 12, 14, 16, 22]
        assert np.all(m.j == 0)
        np.testing.assert_allclose(np.sort(m.A), np.sort([0.5, 0.5, 1.0, 1.0, 2.0, 2.0]), rtol=1e-15)


def test_two_points_self_and_mutual_faces(orc):
    # Two generators on the x axis of a 2 x 1 x 1 box at x = 0.5 and 1.5:
    # each cell is a unit cube; the two mutual faces (direct and through the
    # periodic wall) and the four self-image faces in y and z.
    pos = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5]])
    m = orc.tessellate(pos, (2, 1, 1), method="brute")
    np.testing.assert_allclose(m.V, [1, 1], rtol=1e-15)
    own = m.face_owner()
    f0 = sorted(zip(m.j[own == 0].tolist(), m.code[own == 0].tolist()))
    # image codes: +-y -> 16, 10; +-z -> 22, 4; the wall image of 1 is kx = -1 -> 12
    assert f0 == [(0, 4), (0, 10), (0, 16), (0, 22), (1, 12), (1, 13)]


def test_periodic_translation_invariance(orc):
    # Shifting every generator by a constant vector (modulo the box) leaves
    # the tessellation unchanged up to rounding.
    box = (1.0, 1.0, 1.0)
    pos = W.jittered_lattice((6, 6, 6), box, seed=3)
    m0 = orc.tessellate(pos, box, method="grid")
    sh = np.array([0.37, 0.81, 0.13])
    pos2 = np.mod(pos + sh, 1.0)
    m1 = orc.tessellate(pos2, box, method="grid")
    np.testing.assert_allclose(m1.V, m0.V, rtol=1e-12)
    # Same neighbour sets (image codes differ where a pair now straddles the wall).
    for i in range(0, m0.n, 17):
        s0 = sorted(m0.j[m0.off[i]:m0.off[i + 1]].tolist())
        s1 = sorted(m1.j[m1.off[i]:m1.off[i + 1]].tolist())
        assert s0 == s1
    np.testing.assert_allclose(np.mod(m1.c - sh, 1.0), np.mod(m0.c, 1.0), atol=1e-12)


def test_certificate_flags_degenerate_lattice(orc):
    # An unjittered cubic lattice has eight generators on every vertex
    # sphere: the certificate must report a zero margin; jitter lifts it.
    pos = W.jittered_lattice((4, 4, 4), (1, 1, 1), jitter=0.0)
    m = orc.tessellate(pos, (1, 1, 1), method="grid", certificate=True)
    assert m.delta_min < 1e-14
    np.testing.assert_allclose(m.V, 1 / 64, rtol=1e-12)
    pos = W.jittered_lattice((4, 4, 4), (1, 1, 1), seed=1)
    m = orc.tessellate(pos, (1, 1, 1), method="grid", certificate=True)
    assert m.delta_min > 1e-10


def test_grid_matches_brute_at_4096(orc):
    pos = W.jittered_lattice((16, 16, 16), (1, 1, 1), seed=1)
    mg = orc.tessellate(pos, (1, 1, 1), method="grid", certificate=True)
    assert mg.delta_min > 1e-12
    # Brute force on a sample of cells (every 37th) via a sub-mesh is not
    # possible (cells depend on all points), so the full brute force runs.
    mb = orc.tessellate(pos, (1, 1, 1), method="brute")
    np.testing.assert_array_equal(mb.j, mg.j)
    np.testing.assert_array_equal(mb.code, mg.code)
    np.testing.assert_allclose(mg.V, mb.V, rtol=1e-13)


def test_slab_cells_centroid_closed_form(orc):
    # Two generators on a line along x in a 2 x 1 x 1 box: both cells are
    # slabs bounded by the bisectors, so each centroid is its slab's middle,
    # generally not the generator.
    for x1 in (1.1, 1.3, 1.62, 1.9):
        pos = np.array([[0.3, 0.5, 0.5], [x1, 0.5, 0.5]])
        m = orc.tessellate(pos, (2, 1, 1), method="brute")
        lo, hi = (0.3 + x1 - 2) / 2, (0.3 + x1) / 2
        np.testing.assert_allclose(m.V, [hi - lo, 2 - (hi - lo)], rtol=1e-14)
        np.testing.assert_allclose(m.c[0], [(lo + hi) / 2, 0.5, 0.5], atol=1e-15)
        np.testing.assert_allclose(m.c[1], [(hi + lo + 2) / 2, 0.5, 0.5], atol=1e-15)

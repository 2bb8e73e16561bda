"""The synthetic input recipe: seeded, of the stated shapes, ranges and
structure (512 km square of structured quads, H ~ U[0.5, 2] m and A ~ U[0.8, 1]
drawn H first, a 10 m/s rotating wind gyre and a 0.1 m/s ocean current at the
CG2 nodes, vertices and curved nodes moved within their amplitude, the 64
batched domain sizes). The generators hold none of the method's arithmetic."""
import math

import numpy as np

from synth_inputs import (WORKLOAD_SEEDS, batched_sizes, curved_nodes, make_domain,
                          named_workload, perturbed_vertices, random_state, uniform_vertices)


def test_domains_are_reproducible_per_seed():
    a, b, c = make_domain(20, 12, 6, 1, seed=3), make_domain(20, 12, 6, 1, seed=3), \
        make_domain(20, 12, 6, 1, seed=4)
    for x, y in ((a.H, b.H), (a.A, b.A), (a.vertices, b.vertices), (a.wind, b.wind)):
        assert np.array_equal(x, y)
    assert not np.array_equal(a.H, c.H)


def test_default_mesh_and_ice_fields():
    d = make_domain(64, 32, 6, 1, seed=5)
    h = 512e3 / 64
    V = d.vertices
    assert V.shape == (2, 65 * 33)
    assert V[0].min() == 0.0 and V[0].max() == 512e3 and V[1].max() == 32 * h
    assert d.H.shape == (1, 64 * 32) and d.A.shape == (1, 64 * 32)
    assert 0.5 <= d.H.min() and d.H.max() <= 2.0 and 0.8 <= d.A.min() and d.A.max() <= 1.0
    # H drawn first, then A, from one stream
    rng = np.random.default_rng(5)
    assert np.array_equal(d.H[0], rng.uniform(0.5, 2.0, 64 * 32))
    assert np.array_equal(d.A[0], rng.uniform(0.8, 1.0, 64 * 32))


def test_wind_gyre_and_ocean_current_at_the_nodes():
    nx, ny = 40, 40
    d = make_domain(nx, ny, 6, 1, seed=1)
    nn = (2 * nx + 1) * (2 * ny + 1)
    assert d.wind.shape == (2, nn) and d.ocean.shape == (2, nn)
    speed = np.hypot(d.wind[0], d.wind[1])
    assert speed.max() <= 10.0 + 1e-12 and speed.max() > 9.99
    # sin(pi x) cos(pi y) vanishes on the left edge and the wind is tangential there
    NX = 2 * nx + 1
    left = np.arange(0, nn, NX)
    assert np.abs(d.wind[0][left]).max() < 1e-12
    o = np.hypot(d.ocean[0], d.ocean[1])
    assert abs(o.max() - 0.1) < 1e-12 and o[nn // 2] < 1e-12   # 0.1 m/s at corners, 0 at centre
    rot = make_domain(nx, ny, 6, 1, seed=1, wind_phase=math.pi / 2).wind
    assert np.allclose(rot[0], -d.wind[1]) and np.allclose(rot[1], d.wind[0])


def test_perturbed_vertices_stay_within_amplitude_on_the_box():
    nx, ny, h, amp = 12, 9, 1000.0, 0.15
    U = uniform_vertices(nx, ny, h)
    P = perturbed_vertices(nx, ny, h, amp=amp, seed=2)
    dmax = np.abs(P - U).max()
    assert 0 < dmax <= amp * h
    ix, iy = np.arange(U.shape[1]) % (nx + 1), np.arange(U.shape[1]) // (nx + 1)
    edge = (ix == 0) | (iy == 0) | (ix == nx) | (iy == ny)
    assert np.array_equal(P[:, edge], U[:, edge])


def test_curved_nodes_within_amplitude_and_corners_are_the_vertices():
    nx, ny, h, amp = 10, 8, 1000.0, 0.15
    N = curved_nodes(nx, ny, h, amp=amp, seed=3)
    NX, NY = 2 * nx + 1, 2 * ny + 1
    ix, iy = np.arange(NX * NY) % NX, np.arange(NX * NY) // NX
    assert np.abs(N[0] - ix * h / 2).max() <= amp * h and np.abs(N[1] - iy * h / 2).max() <= amp * h
    d = make_domain(nx, ny, 6, 1, seed=4, h=h, curved=amp)
    corner = (iy % 2 == 0) & (ix % 2 == 0)
    assert np.array_equal(d.vertices, d.nodes[:, corner])


def test_batched_sizes_and_named_workloads():
    sizes, phases = batched_sizes()
    assert len(sizes) == 64 and sizes[0] == 64 and sizes[-1] == 512
    assert all(64 <= s <= 512 for s in sizes) and len(phases) == 64
    assert batched_sizes() == (sizes, phases)
    (d,) = named_workload("32x32-dg1")
    assert (d.nx, d.ny, d.n_s, d.n_a) == (32, 32, 3, 1) and d.meta["h"] == 10e3
    assert d.meta["seed"] == WORKLOAD_SEEDS["32x32-dg1"]


def test_random_state_is_at_rest_on_the_boundary():
    nx, ny = 9, 7
    v, S = random_state(nx, ny, 6, seed=8)
    NX, NY = 2 * nx + 1, 2 * ny + 1
    ix, iy = np.arange(NX * NY) % NX, np.arange(NX * NY) // NX
    bnd = (ix == 0) | (iy == 0) | (ix == NX - 1) | (iy == NY - 1)
    assert v.shape == (2, NX * NY) and S.shape == (3, 6, nx * ny)
    assert (v[:, bnd] == 0).all() and np.abs(v[:, ~bnd]).max() > 0 and np.abs(S).max() > 0

"""The seeded input generators: deterministic, the advertised shapes and ranges."""
import math

import numpy as np

import workloads as W


def test_ricker_peak_and_delay():
    dt, f0 = 20e-9, 2.5e6
    w = W.ricker(f0, dt, 400)
    assert w.dtype == np.float32
    k = int(np.argmax(w))
    assert abs(k * dt - 1.5 / f0) <= dt
    assert abs(float(w[k]) - 1.0) < 1e-3
    assert abs(float(w[0])) < 1e-6


def test_rodgauss512_deterministic_and_ranges():
    a = W.c2_medium(20, n_tx=16, nt=50)
    b = W.c2_medium(20, n_tx=16, nt=50)
    assert np.array_equal(a.c, b.c) and np.array_equal(a.rho, b.rho)
    c = W.c2_medium(21, n_tx=16, nt=50)
    assert not np.array_equal(a.c, c.c)
    g = a.geom
    assert (g.nx, g.nz, g.n_tx, g.n_rcv) == (512, 512, 16, 128)
    assert a.c.dtype == np.float32 and a.c.shape == (512, 512)
    assert 1440 < a.c.min() and a.c.max() < 1650
    assert 969 <= a.rho.min() and a.rho.max() <= 1031
    # array on row 20 at pitch 3, transmitters spread over it
    cells = g.rcv[0]
    assert np.all(cells // 512 == 20)
    assert np.all(np.diff(cells % 512) == 3)
    assert g.src[0] == cells[0] and g.src[-1] == cells[-1]


def test_disc128():
    m = W.c1_small()
    g = m.geom
    assert (g.nx, g.nt, g.n_tx, g.n_rcv) == (128, 1000, 1, 32)
    assert m.c.min() == 1500 and m.c.max() == 1540
    inside = np.sum(m.c == 1500)
    assert abs(inside - math.pi * 15 ** 2) < 30
    assert np.all(W.c1_small(partner=True).c == 1540)


def test_uneven_batch_recipe():
    media = W.c4_batch(40, n_media=8, steps_scale=0.01)
    for m in media:
        g = m.geom
        assert 256 <= g.nx <= 768 and g.nx == g.nz
        assert 8 <= g.n_tx <= 32 and g.n_tx <= g.n_rcv
        assert g.n_rcv == min(128, (g.nx - 41) // 3 + 1)
    again = W.c4_batch(40, n_media=8, steps_scale=0.01)
    assert all(np.array_equal(a.c, b.c) for a, b in zip(media, again))

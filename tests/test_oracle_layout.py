"""Pins for the oracle's scene storage order (Morton order of the means):
bit interleaving against hand values, quantisation endpoints and the
non-finite / flat-axis cases, and a brute-force comparison of whole orders
(CPU only)."""
import numpy as np

from oracle import layout


def test_interleave_hand_values():
    assert layout.interleave(1, 0, 0) == 1
    assert layout.interleave(0, 1, 0) == 2
    assert layout.interleave(0, 0, 1) == 4
    assert layout.interleave(2, 0, 0) == 8
    assert layout.interleave(1023, 1023, 1023) == (1 << 30) - 1
    assert layout.interleave(0b11, 0b01, 0b10) == 0b101011
    # a larger coordinate in the most significant axis bit orders after
    assert layout.interleave(0, 0, 512) > layout.interleave(1023, 1023, 511)


def test_quantise_endpoints_and_special_values():
    m = np.array([[0.0, 1.0, 0.5, np.nan], [2.0, 2.0, 2.0, 2.0], [-1.0, 3.0, np.inf, 0.0]],
                 dtype=np.float32)
    q = layout.quantise(m)
    assert q[0].tolist() == [0, 1023, 512, 1023]       # lo -> 0, hi -> 1023 (clamped), NaN -> 1023
    assert q[1].tolist() == [0, 0, 0, 0]               # flat axis
    assert q[2].tolist() == [0, 1023, 1023, 256]       # inf ignored for the box, then 1023


def test_order_brute_force():
    rng = np.random.default_rng(4)
    m = rng.normal(size=(3, 300)).astype(np.float32)
    m[:, 50:60] = m[:, 40:41]  # equal codes keep the original order
    order = layout.morton_order(m)
    q = layout.quantise(m)
    codes = [layout.interleave(*[int(q[a][i]) for a in range(3)]) for i in range(300)]
    want = sorted(range(300), key=lambda i: (codes[i], i))
    assert order.tolist() == want
    # neighbours in the order are close in space on average
    d_sorted = np.linalg.norm(np.diff(m[:, order], axis=1), axis=0).mean()
    d_random = np.linalg.norm(np.diff(m, axis=1), axis=0).mean()
    assert d_sorted < 0.5 * d_random

"""Host-side checks of arithmetic the kernels rely on (no GPU needed).

divmod_u32 in csrc/k_cub_fwd.hip computes floor(v / n) for v, n < 2^32 as the
truncated double-precision product v * (1 / n) followed by one correction
step in either direction.  The double quotient is within 2^-20 of v / n, so a
single step suffices; this test replays the same IEEE double arithmetic."""
import numpy as np


def _divmod(v: int, n: int):
    inv = 1.0 / float(n)
    q = int(float(v) * inv)
    r = v - q * n
    if r >= n:
        q, r = q + 1, r - n
    if r < 0:
        q, r = q - 1, r + n
    return q, r


def test_double_divmod_is_exact():
    g = np.random.default_rng(7)
    cases = [(v, n) for n in (1, 2, 3, 7, 64, 128, 192, 255, 1023, 2 ** 20 + 1, 2 ** 31 - 1, 2 ** 32 - 1)
             for v in (0, 1, n - 1, n, n + 1, 2 * n - 1, 2 ** 24 - 1, 2 ** 24 + 1, 2 ** 31, 2 ** 32 - 1) if 0 <= v < 2 ** 32]
    for _ in range(20000):
        n = int(g.integers(1, 2 ** 32))
        cases.append((int(g.integers(0, 2 ** 32)), n))
        n = int(g.integers(1, 4096))
        cases.append((int(g.integers(0, 2 ** 32)), n))
        k = int(g.integers(0, 2 ** 20))
        cases.append((min(max(k * n + int(g.integers(-1, 2)), 0), 2 ** 32 - 1), n))  # next to a multiple
    for v, n in cases:
        assert _divmod(v, n) == (v // n, v % n), (v, n)

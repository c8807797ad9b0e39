"""Order in which iGNNS draws its random restart nodes.

The paper draws "a random node" whenever the climb reaches a local maximum
and also when a drawn node fails the expansion test (Section 3).  It does not
say how.  Reading used here: nodes are drawn *without replacement* along a
keyed pseudo-random permutation of [0, n), skipping nodes already evaluated.
This makes the search a deterministic function of (graph, query, seed, key),
and with an unlimited budget every node is eventually evaluated.

The permutation is a full-period linear congruential sequence modulo
m = 2^ceil(log2 n):  x_{t+1} = (a * x_t + c) mod m.  By the Hull-Dobell
theorem the period is m iff c is odd and a = 1 (mod 4) (for m >= 4), so
x_0 .. x_{m-1} visit every residue once; values >= n are skipped
(cycle-walking).  The parameters (a, c, x_0) are drawn from the SplitMix64
generator (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014):

    s  = seed XOR first_output(SplitMix64 seeded with key)
    r0, r1, r2 = the first three outputs of SplitMix64 seeded with s
    a  = 4 * (r0 mod m/4) + 1,  c = 2 * (r1 mod m/2) + 1,  x_0 = r2 mod m
    (for m <= 2: a = c = 1)

The key of an inserted point is its global id; the key of a read-only query
is 2^62 plus its query sequence number.
"""

from __future__ import annotations

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_next(state: int) -> tuple[int, int]:
    """One step of SplitMix64: returns (new_state, output)."""
    state = (state + GOLDEN_GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def modulus_for(n: int) -> int:
    m = 1
    while m < n:
        m <<= 1
    return m


def restart_params(n: int, seed: int, key: int) -> tuple[int, int, int, int]:
    """(m, a, c, x0) of the restart permutation for snapshot size n."""
    _, hk = splitmix64_next(key & MASK64)
    s = (seed ^ hk) & MASK64
    s, r0 = splitmix64_next(s)
    s, r1 = splitmix64_next(s)
    s, r2 = splitmix64_next(s)
    m = modulus_for(n)
    if m <= 2:
        a, c = 1, 1
    else:
        a = 4 * (r0 % (m // 4)) + 1
        c = 2 * (r1 % (m // 2)) + 1
    x0 = r2 % m
    return m, a, c, x0


class RestartOrder:
    """Walks the permutation; ``next_unvisited`` returns the next node id
    that is < n and not in ``visited``, or None once all m positions are
    used."""

    def __init__(self, n: int, seed: int, key: int):
        self.n = n
        self.m, self.a, self.c, self.x = restart_params(n, seed, key)
        self.t = 0          # number of positions consumed

    def next_unvisited(self, visited) -> int | None:
        while self.t < self.m:
            x = self.x
            self.x = (self.a * self.x + self.c) % self.m
            self.t += 1
            if x < self.n and x not in visited:
                return x
        return None

    def full_sequence(self) -> list[int]:
        """All m values x_0 .. x_{m-1}; only valid before the first draw."""
        if self.t != 0:
            raise RuntimeError("full_sequence must be called before drawing")
        out, x = [], self.x
        for _ in range(self.m):
            out.append(x)
            x = (self.a * x + self.c) % self.m
        return out

"""Replay of the direction-optimising rule -- TEST INFRASTRUCTURE ONLY.

Beamer, Asanovic and Patterson, "Direction-Optimizing Breadth-First Search"
(SC 2012), which the paper cites as the origin of pull BFS (Sec. "An Example
Design-Space Exploration: From Push to Pull BFS").  With m_f the out-edges of
the frontier, m_u the in-edges of the unvisited vertices and n_f the frontier
size, the search starts top-down and
  * switches top-down -> bottom-up when m_f > m_u / alpha,
  * switches bottom-up -> top-down when n_f < n / beta and the frontier
    shrank since the previous level,
with the published constants alpha = 14, beta = 24.
"""
from __future__ import annotations

ALPHA = 14
BETA = 24
PUSH, PULL = 0, 1


def replay(n: int, nF, eF, eU, alpha: int = ALPHA, beta: int = BETA):
    """Direction used at each level, given the per-level counts."""
    out = []
    d = PUSH
    prev_nf = None
    for k in range(len(nF)):
        if d == PUSH:
            if eF[k] * alpha > eU[k]:
                d = PULL
        else:
            shrinking = prev_nf is not None and nF[k] < prev_nf
            if nF[k] * beta < n and shrinking:
                d = PUSH
        out.append(d)
        prev_nf = nF[k]
    return out

"""Algorithmic HBM bytes of one level step, per variant.

These are the bytes the method itself must move, not what the hardware
fetches: a status lookup in a bitmap counts 1/8 byte, a CSR offset pair 8
bytes, a column id 4 bytes.  Inputs are the per-level counts the library
reports (bfs_stats per-level arrays):

  nF   |F_k|              eF   out-edges of F_k
  nU   |U_{k-1}|, the unvisited set the step searches (before F_{k+1})
  nN   |F_{k+1}|          scan edges the step examined (pull: early-exit scan)
  n    vertices

Per variant (p = 4 when parents are written, else 0):
  push, queue in (thread/block)   4nF + 8nF + 4eF + eF/8 + (8+p)nN + nN/8
  push, merge path                as above + 8nF (degree scan written and read)
  push, bitmap in, atomic         n/8 + 8nF + 4eF + eF/8 + (8+p)nN + nN/8
  push, atomic-free (q or b in)   [4nF | n/8] + 8nF + 4eF + eF/8 + (4+p)nN
                                  + update pass: n/8 + 4nU + 2n/8 + 4nN
  pull, bitmap                    n/8 + 8nU + 4scan + scan/8 + 2n/8 + (8+p)nN
  pull, visited as frontier       n/8 + 8nU + 4scan + scan/8 + n/8 + (8+p)nN
                                  + merge pass 3n/8
  push, three visited arrays      2n/8 (F = P_k AND NOT P_{k-1}) + 8nF + 4eF + eF/8
                                  + (4+p)nN + update pass: n/8 + 4nU + 3n/8 + 4nN
  push, advance then filter       20nF (queue, offsets, degree scan) + 4eF + 8eF (list
                                  written) + 8eF (read back) + eF/8 + (8+p)nN + nN/8
  (bitmap frontier)               2n/8 + 16nF + 4W (word scan) + the same per edge and nN
  push, best-effort dedup         12nF + 4eF + eF/8 + (4+p)nN (depth, parent of each candidate;
                                  about nN of them) + 16nN (list written, read back) + nN/8
                                  (filter's visited test) + 4nN + nN/8 (queue, next bitmap)
"""
from __future__ import annotations

from . import _lib as L


def step_bytes(variant: int, n: int, nF: int, eF: int, nU: int, nN: int, scan: int, parents: bool = False) -> float:
    p = 4 if parents else 0
    bm = n / 8.0
    if variant in (L.PUSH_Q_THREAD, L.PUSH_Q_BLOCK, L.PUSH_Q_MERGE):
        b = 12.0 * nF + 4.0 * eF + eF / 8.0 + (8 + p) * nN + nN / 8.0
        if variant == L.PUSH_Q_MERGE:
            b += 8.0 * nF
        return b
    if variant == L.PUSH_B_ATOMIC:
        return bm + 8.0 * nF + 4.0 * eF + eF / 8.0 + (8 + p) * nN + nN / 8.0
    if variant in (L.PUSH_B_NOATOMIC, L.PUSH_Q_NOATOMIC):
        head = bm if variant == L.PUSH_B_NOATOMIC else 4.0 * nF
        return head + 8.0 * nF + 4.0 * eF + eF / 8.0 + (4 + p) * nN + bm + 4.0 * nU + 2 * bm + 4.0 * nN
    if variant == L.PULL_B:
        return bm + 8.0 * nU + 4.0 * scan + scan / 8.0 + 2 * bm + (8 + p) * nN
    if variant == L.PULL_VIS:  # probes read the visited bitmap; merge pass reads next, updates visited
        return bm + 8.0 * nU + 4.0 * scan + scan / 8.0 + bm + (8 + p) * nN + 3 * bm
    if variant == L.PUSH_Q_FILTER:  # neighbours and sources go through the temporary list
        return 20.0 * nF + 4.0 * eF + 16.0 * eF + eF / 8.0 + (8 + p) * nN + nN / 8.0
    if variant == L.PUSH_B_FILTER:  # word weights scanned, then the same list
        return 2 * bm + 16.0 * nF + 4.0 * (n / 64.0) + 4.0 * eF + 16.0 * eF + eF / 8.0 + (8 + p) * nN + nN / 8.0
    if variant == L.PUSH_Q_DEDUP:  # atomic-free advance: nN candidates (depth, parent, list entry), then the filter
        return 12.0 * nF + 4.0 * eF + eF / 8.0 + (4 + p) * nN + 8.0 * nN + 8.0 * nN + nN / 8.0 + 4.0 * nN + nN / 8.0
    if variant == L.PUSH_P3:  # frontier from two visited arrays; update also writes P_{k-1}
        return 2 * bm + 8.0 * nF + 4.0 * eF + eF / 8.0 + (4 + p) * nN + bm + 4.0 * nU + 3 * bm + 4.0 * nN
    raise ValueError(variant)


def reset_bytes(n: int, parents: bool = False) -> float:
    return 4.0 * n * (2 if parents else 1) + 4 * n / 8.0


def level_bytes(stats: dict, n: int, parents: bool = False):
    """Per-level algorithmic bytes of a finished search (stats with per-level
    arrays, as returned by bfs_levels(..., level_stats=True))."""
    out = []
    k = int(stats["num_levels"])
    for i in range(k):
        nU_before = int(stats["unvisited"][i])  # unvisited after F_i was found = searched by step i
        out.append(step_bytes(int(stats["variant"][i]), n, int(stats["frontier"][i]),
                              int(stats["frontier_edges"][i]), nU_before, int(stats["next"][i]),
                              int(stats["scanned"][i]), parents))
    return out


MS_PLANES = 8  # depth bit planes per window of the multi-source search


def ms_rel(k: int) -> int:
    """Relative depth stored by level k's discoveries (windows of 255 levels)."""
    return k % ((1 << MS_PLANES) - 1) + 1


def ms_step_bytes(pull: bool, n: int, k: int, nf: int, unvis: int, scan: int, hits: int, found: int,
                  pscan: int = 0, pact: int = 0) -> float:
    """One level k of the 64-lane multi-source search (u64 words per vertex).

    Both directions clear the dead frontier buffer (8n) and record each found
    vertex as a visited-word write plus a read-modify-write of the depth
    planes the relative depth sets (16 bytes per set bit).
      bottom-up: 8n visited + 8n next words + n/8 next bitmap + 8 per unvis
                 (csc_ptr pair) + 4 per scanned in-edge + 1/8 per probe of the
                 frontier bitmap + 8 per gathered frontier word (hits)
      top-down : n/8 frontier bitmap + 16 per frontier vertex (word, row_ptr
                 pair) + 12 per scanned edge (target id, its visited word)
                 + 8 per found vertex (its next word) + update pass: 8n next
                 words + n/8 next bitmap + 8 per found (visited read)
      split bottom-up (pact > 0 or pscan > 0): the bottom-up terms over the
                 pulled in-edges (scan - pscan), plus 8 per unvis (the pushed
                 next word read as the start of the OR) and the push: n/8
                 frontier bitmap + 16 per pushing vertex (word, row_ptr pair)
                 + 12 per pushed edge (target id, its visited word)
    nf = frontier vertices, unvis = vertices missing some lane (bottom-up),
    hits = in-edges whose source is in the frontier, found = vertices with a
    new lane, pscan / pact = edges and vertices of a split level's push."""
    disc = found * (8.0 + 16.0 * bin(ms_rel(k)).count("1"))
    if pull:
        split = 8.0 * unvis + n / 8.0 + 16.0 * pact + 12.0 * pscan if (pscan or pact) else 0.0
        return (8.0 * n + 8.0 * n + 8.0 * n + n / 8.0 + 8.0 * unvis + 4.125 * (scan - pscan) + 8.0 * hits + disc
                + split)
    return 8.0 * n + n / 8.0 + 16.0 * nf + 12.0 * scan + 8.0 * found + 8.0 * n + n / 8.0 + 8.0 * found + disc


def ms_tile_bytes(n: int, k: int, unvis: int, scan_light: int, hits_light: int, found: int,
                  split: bool = False) -> float:
    """The bottom-up tile kernel alone: the dense per-vertex part (8n visited
    read, 8n next written, 8n dead buffer cleared, n/8 next bitmap, 8 per
    unvis for the csc_ptr pair), the light vertices' in-edges (4 per column id
    + 1/8 per bitmap probe), their gathered frontier words (8 each) and the
    discoveries (visited write + plane updates).  The heavy kernel's edges and
    gathers are excluded (scan_light = scanned - scanned_aux, hits_light =
    hits - hits_aux); on a split level so are the push's edges (scan_light
    also less scanned_push), and each unvis vertex reads its pushed next word
    (8 more)."""
    disc = found * (8.0 + 16.0 * bin(ms_rel(k)).count("1"))
    return (24.0 * n + n / 8.0 + (16.0 if split else 8.0) * unvis + 4.125 * scan_light + 8.0 * hits_light
            + disc)


def ms_tile_level_bytes(stats: dict, n: int):
    """ms_tile_bytes for every bottom-up level (split or not) of a bfs_multi
    run (None for top-down levels)."""
    out = []
    k = 0
    for i in range(int(stats["num_levels"])):
        var = int(stats["variant"][i])
        if var in (L.PULL_B, L.MS_SPLIT):
            push = int(stats["scanned_push"][i]) if "scanned_push" in stats else 0
            out.append(ms_tile_bytes(n, k, int(stats["unvisited"][i]),
                                     int(stats["scanned"][i]) - int(stats["scanned_aux"][i]) - push,
                                     int(stats["frontier_ld2"][i]) - int(stats["hits_aux"][i]),
                                     int(stats["frontier_ld"][i]), split=var == L.MS_SPLIT))
        else:
            out.append(None)
        k = 0 if int(stats["next"][i]) == 0 else k + 1
    return out


def ms_level_bytes(stats: dict, n: int):
    """Per-level bytes of a bfs_multi run with level stats (one group of up to
    64 lanes: the level index restarts at 0 for each group)."""
    out = []
    k = 0
    for i in range(int(stats["num_levels"])):
        pull = int(stats["variant"][i]) in (L.PULL_B, L.MS_SPLIT)
        split = int(stats["variant"][i]) == L.MS_SPLIT
        out.append(ms_step_bytes(pull, n, k, int(stats["frontier"][i]), int(stats["unvisited"][i]),
                                 int(stats["scanned"][i]), int(stats["frontier_ld2"][i]),
                                 int(stats["frontier_ld"][i]),
                                 int(stats["scanned_push"][i]) if split else 0,
                                 int(stats["push_sources"][i]) if split else 0))
        k = 0 if int(stats["next"][i]) == 0 else k + 1
    return out


def ms_fixed_bytes(n: int, lanes: int, planes: int) -> float:
    """Per group outside the levels: zeroing visited, two frontier buffers and
    the frontier bitmap (24n + n/8), zeroing the planes in use (8n each), and
    the output pass (8n visited + 8n per plane read, 4 bytes per (lane,
    vertex) written, each row once)."""
    return 24.0 * n + n / 8.0 + 8.0 * n * planes + 8.0 * n + 8.0 * n * planes + 4.0 * lanes * n


def batch_bytes(total_n: int, reached: int, comp_edges: int) -> float:
    """The batched launch over all its instances: every depth written once
    (4 per vertex), and per reached vertex its row_ptr pair read once (8) and
    its queue slot written and read (8), and its out-edges' column ids read
    once (4 per edge of the traversed components, comp_edges) -- the
    push-queue bytes per level summed over the search, with the visited
    status in on-chip memory.  Bottom-up levels read fewer column ids (early
    exit), so this is the top-down cost of the method."""
    return 4.0 * total_n + 16.0 * reached + 4.0 * comp_edges

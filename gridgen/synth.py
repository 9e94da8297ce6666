"""Seeded synthetic power-grid inputs shared by the CPU oracle and the GPU library.

This module holds input generation only: bus placement, topology, branch
parameters, the partition into areas, true bus states, snapshot drift and the
standard-normal noise draws.  It holds none of the estimation arithmetic: no
branch admittance, no measurement function h(x), no Jacobian, no Gauss-Newton
step.  A consumer builds measurements as z = h(x_true) + sigma * eps with its
own h; `eps` (the random numbers) come from here so both sides see the same
draws.

The generator rule follows the workload description of the paper's benchmark
grids (PEGASE-2869, PEGASE-9241, ACTIVSg10k, Section 5.1) at their bus and
branch counts; those case files are not reproduced, these synthetic grids stand
in for them:

* buses uniform in the unit square;
* an exact Euclidean minimum spanning tree (Kruskal on the Delaunay edges);
* then nearest-neighbour chords, one per visited bus, visiting the buses in a
  seeded random permutation (cycling), each adding a branch to its nearest bus
  that is not yet adjacent, until the branch count is reached;
* x = 0.01 + 0.19 * length, r = x * U(0.05, 0.3), total line charging
  b = U(0, 0.04) (per unit);
* true state |V| ~ U(0.95, 1.05), theta = -0.3 * (distance to bus 0) +
  N(0, 0.01) rad, theta of the slack bus 0 is 0;
* measurements: |V| at every bus (sigma 0.004), P and Q injection at every bus
  (sigma 0.01), P and Q flow at both ends of every branch (sigma 0.008);
* partition: farthest-point seeds (first seed bus 0), then breadth-first growth
  by hop count; "plain" lets all areas grow from one FIFO queue, "balanced"
  lets the currently smallest area claim the next bus.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.spatial import Delaunay, cKDTree

# Measurement type codes.  The order of the measurement vector built by
# `measurement_set` is: VM at all buses, PINJ at all buses, QINJ at all buses,
# PF, QF, PT, QT at all branches.
VM, PINJ, QINJ, PF, QF, PT, QT = range(7)
TYPE_NAMES = ("VM", "PINJ", "QINJ", "PF", "QF", "PT", "QT")

SIGMA_VM = 0.004
SIGMA_INJ = 0.01
SIGMA_FLOW = 0.008

# Snapshot drift (per step): |V| jitter N(0, 0.003), theta jitter N(0, 0.005).
DRIFT_VM = 0.003
DRIFT_VA = 0.005

# (buses, branches, areas, partition mode) of the four synthetic workloads.
CONFIGS = {
    "c0": (30, 41, 3, "plain"),
    "c1": (2869, 4582, 8, "balanced"),
    "c2": (9241, 16049, 32, "plain"),
    "c3": (10000, 12706, 16, "plain"),
}

SLACK_BUS = 0


@dataclasses.dataclass
class Grid:
    pos: np.ndarray        # [n_bus, 2] float64
    br_from: np.ndarray    # [n_branch] int32
    br_to: np.ndarray      # [n_branch] int32
    br_r: np.ndarray       # [n_branch] float64, series resistance (p.u.)
    br_x: np.ndarray       # [n_branch] float64, series reactance (p.u.)
    br_b: np.ndarray       # [n_branch] float64, total line charging (p.u.)
    vm: np.ndarray         # [n_bus] float64, true |V|
    va: np.ndarray         # [n_bus] float64, true theta (rad), va[0] == 0
    bus_area: np.ndarray   # [n_bus] int32
    n_area: int
    slack: int = SLACK_BUS

    @property
    def n_bus(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_branch(self) -> int:
        return int(self.br_from.shape[0])


def _emst_edges(pos: np.ndarray) -> np.ndarray:
    """Exact Euclidean MST: Kruskal restricted to Delaunay edges."""
    n = pos.shape[0]
    if n == 2:
        return np.array([[0, 1]], dtype=np.int64)
    tri = Delaunay(pos)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    w = np.linalg.norm(pos[e[:, 0]] - pos[e[:, 1]], axis=1)
    g = coo_matrix((w, (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    t = minimum_spanning_tree(g).tocoo()
    out = np.stack([t.row, t.col], axis=1).astype(np.int64)
    out.sort(axis=1)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def _add_chords(pos: np.ndarray, edges: list, n_branch: int, rng) -> list:
    n = pos.shape[0]
    if n_branch > n * (n - 1) // 2:
        raise ValueError("more branches than bus pairs")
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    tree = cKDTree(pos)
    perm = rng.permutation(n)
    k = 0
    while len(edges) < n_branch:
        u = int(perm[k % n])
        k += 1
        if len(adj[u]) >= n - 1:
            continue
        kk = len(adj[u]) + 2
        while True:
            _, idx = tree.query(pos[u], k=min(kk, n))
            idx = np.atleast_1d(idx)
            cand = [int(v) for v in idx if v != u and v not in adj[u]]
            if cand:
                v = cand[0]
                break
            kk *= 2
        a, b = (u, v) if u < v else (v, u)
        edges.append((a, b))
        adj[a].add(b)
        adj[b].add(a)
    return edges


def _adjacency(n_bus: int, br_from, br_to) -> list:
    adj = [[] for _ in range(n_bus)]
    for f, t in zip(br_from.tolist(), br_to.tolist()):
        adj[f].append(t)
        adj[t].append(f)
    return [sorted(set(a)) for a in adj]


def farthest_point_seeds(pos: np.ndarray, n_area: int) -> list:
    seeds = [0]
    mind = np.linalg.norm(pos - pos[0], axis=1)
    for _ in range(n_area - 1):
        s = int(np.argmax(mind))  # first maximum: lowest index on ties
        seeds.append(s)
        mind = np.minimum(mind, np.linalg.norm(pos - pos[s], axis=1))
    return seeds


def partition(pos, br_from, br_to, n_area: int, mode: str = "plain") -> np.ndarray:
    """Area of every bus: farthest-point seeds, then BFS growth by hop count."""
    n = pos.shape[0]
    adj = _adjacency(n, np.asarray(br_from), np.asarray(br_to))
    seeds = farthest_point_seeds(pos, n_area)
    area = np.full(n, -1, dtype=np.int32)
    for k, s in enumerate(seeds):
        area[s] = k
    if mode == "plain":
        queue = list(seeds)
        head = 0
        while head < len(queue):
            u = queue[head]
            head += 1
            for v in adj[u]:
                if area[v] < 0:
                    area[v] = area[u]
                    queue.append(v)
    elif mode == "balanced":
        queues = [[s] for s in seeds]
        heads = [0] * n_area
        sizes = [1] * n_area
        while True:
            best = -1
            for k in range(n_area):
                if heads[k] < len(queues[k]) and (best < 0 or sizes[k] < sizes[best]):
                    best = k
            if best < 0:
                break
            k = best
            claimed = False
            while heads[k] < len(queues[k]) and not claimed:
                u = queues[k][heads[k]]
                for v in adj[u]:
                    if area[v] < 0:
                        area[v] = k
                        queues[k].append(v)
                        sizes[k] += 1
                        claimed = True
                        break
                if not claimed:
                    heads[k] += 1
    else:
        raise ValueError(mode)
    if (area < 0).any():
        raise ValueError("grid is not connected")
    return area


def make_grid(n_bus: int, n_branch: int, n_area: int, seed: int = 0,
              mode: str = "plain") -> Grid:
    """Build a seeded synthetic grid with its true state and partition."""
    if n_branch < n_bus - 1:
        raise ValueError("need at least n_bus - 1 branches for a connected grid")
    rng = np.random.default_rng(seed)
    pos = rng.random((n_bus, 2))
    edges = [tuple(map(int, e)) for e in _emst_edges(pos)]
    edges = _add_chords(pos, edges, n_branch, rng)
    e = np.asarray(edges, dtype=np.int64)
    length = np.linalg.norm(pos[e[:, 0]] - pos[e[:, 1]], axis=1)
    x = 0.01 + 0.19 * length
    r = x * rng.uniform(0.05, 0.3, size=len(e))
    b = rng.uniform(0.0, 0.04, size=len(e))
    vm = rng.uniform(0.95, 1.05, size=n_bus)
    va = -0.3 * np.linalg.norm(pos - pos[SLACK_BUS], axis=1) + rng.normal(0.0, 0.01, size=n_bus)
    va[SLACK_BUS] = 0.0
    br_from = e[:, 0].astype(np.int32)
    br_to = e[:, 1].astype(np.int32)
    bus_area = partition(pos, br_from, br_to, n_area, mode)
    return Grid(pos=pos, br_from=br_from, br_to=br_to, br_r=r, br_x=x, br_b=b,
                vm=vm, va=va, bus_area=bus_area, n_area=n_area)


def make_config(name: str, seed: int = 0) -> Grid:
    n_bus, n_branch, n_area, mode = CONFIGS[name]
    return make_grid(n_bus, n_branch, n_area, seed=seed, mode=mode)


def measurement_set(n_bus: int, n_branch: int):
    """Full measurement set: (type, bus-or-branch index, sigma) per row."""
    types = np.concatenate([
        np.full(n_bus, VM), np.full(n_bus, PINJ), np.full(n_bus, QINJ),
        np.full(n_branch, PF), np.full(n_branch, QF),
        np.full(n_branch, PT), np.full(n_branch, QT)]).astype(np.int32)
    at = np.concatenate([np.arange(n_bus)] * 3 + [np.arange(n_branch)] * 4).astype(np.int32)
    sigma = np.concatenate([
        np.full(n_bus, SIGMA_VM), np.full(2 * n_bus, SIGMA_INJ),
        np.full(4 * n_branch, SIGMA_FLOW)]).astype(np.float64)
    return types, at, sigma


def drift_states(vm0, va0, n_snap: int, rng, slack: int = SLACK_BUS):
    """Snapshot 0 is the base state; snapshot s = snapshot s-1 + jitter."""
    n = vm0.shape[0]
    vm = np.empty((n_snap, n))
    va = np.empty((n_snap, n))
    vm[0] = vm0
    va[0] = va0
    for s in range(1, n_snap):
        vm[s] = vm[s - 1] + rng.normal(0.0, DRIFT_VM, size=n)
        va[s] = va[s - 1] + rng.normal(0.0, DRIFT_VA, size=n)
        va[s, slack] = 0.0
    return vm, va


def noise_draws(n_snap: int, n_meas: int, rng) -> np.ndarray:
    """Standard-normal draws eps[s, i]; measurement noise is sigma_i * eps[s, i]."""
    return rng.standard_normal((n_snap, n_meas))


@dataclasses.dataclass
class Batch:
    grid: Grid
    meas_type: np.ndarray
    meas_at: np.ndarray
    meas_sigma: np.ndarray
    vm_true: np.ndarray   # [n_snap, n_bus]
    va_true: np.ndarray   # [n_snap, n_bus]
    eps: np.ndarray       # [n_snap, n_meas] standard normal


def make_batch(grid: Grid, n_snap: int, seed: int = 0) -> Batch:
    """Snapshots of one grid: drifted true states and fresh noise per snapshot.

    Seeds derive from SeedSequence(seed): child 0 drives the drift, child 1
    the noise, so the same (grid, seed) always yields the same batch.
    """
    t, a, s = measurement_set(grid.n_bus, grid.n_branch)
    ss = np.random.SeedSequence(seed).spawn(2)
    vm, va = drift_states(grid.vm, grid.va, n_snap, np.random.default_rng(ss[0]), grid.slack)
    eps = noise_draws(n_snap, t.shape[0], np.random.default_rng(ss[1]))
    return Batch(grid, t, a, s, vm, va, eps)


def make_chains(grid: Grid, n_chain: int, chain_len: int, seed: int):
    """Independent drift chains from the base state (training / held-out sets).

    Returns vm, va of shape [n_chain * chain_len, n_bus] and eps of shape
    [n_chain * chain_len, n_meas]; chain c uses SeedSequence(seed + c).
    """
    t, _, _ = measurement_set(grid.n_bus, grid.n_branch)
    vms, vas, epss = [], [], []
    for c in range(n_chain):
        ss = np.random.SeedSequence(seed + c).spawn(2)
        vm, va = drift_states(grid.vm, grid.va, chain_len + 1, np.random.default_rng(ss[0]), grid.slack)
        vms.append(vm[1:])
        vas.append(va[1:])
        epss.append(noise_draws(chain_len, t.shape[0], np.random.default_rng(ss[1])))
    return np.concatenate(vms), np.concatenate(vas), np.concatenate(epss)


def grid_stats(grid: Grid) -> dict:
    """Counts printed beside every workload: N, B, m, n, K, area sizes, boundary."""
    f, t, ar = grid.br_from, grid.br_to, grid.bus_area
    cut = ar[f] != ar[t]
    bnd = np.zeros(grid.n_bus, dtype=bool)
    bnd[f[cut]] = True
    bnd[t[cut]] = True
    sizes = np.bincount(ar, minlength=grid.n_area)
    n_gamma = 2 * int(bnd.sum()) - int(bnd[grid.slack])
    return {
        "N": grid.n_bus, "B": grid.n_branch, "K": grid.n_area,
        "m": 3 * grid.n_bus + 4 * grid.n_branch, "n": 2 * grid.n_bus - 1,
        "area_min": int(sizes.min()), "area_max": int(sizes.max()),
        "cut_branches": int(cut.sum()), "boundary_buses": int(bnd.sum()),
        "boundary_frac": float(bnd.mean()), "n_gamma": n_gamma,
    }

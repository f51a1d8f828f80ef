"""Tent pitching for the oracle (section "Mesh generation by tent pitching").

The paper fixes: the front is a P1 function given by one time per vertex; a tent moves
one vertex up; its projection is the vertex patch; vertices at graph distance >= 2 can
move independently; the advance is limited by causality (|grad phi| < sqrt(eps mu)),
and the experiments bound the front slope by 1/(2c).  The paper defers the pitching
algorithm to earlier work, so the concrete rule below is a documented reading that both
implementations follow:

  per element T:   k_T = sigma sqrt(eps_T mu_T) / min_i sum_{j != i} |grad lambda_j^T|
  per edge (v,w):  k_vw = min over elements T containing the edge of k_T
  repeat: take the vertex v with the smallest (tau_v, v) below t_end;
          t_plus = min over neighbours w of (tau_w + k_vw);
          t_new  = min(t_end, Q floor(t_plus / Q - 1e-3)),  Q = 2^-24;
          emit tent (v, tau_v, t_new) in layer 1 + max(last layer of v and of its
          neighbours); tau_v = t_new.

A second ordering ("colour") moves the vertices in another order, which the paper allows
(any order that keeps causality gives valid tents):
  colour the vertex graph greedily (ids ascending, each vertex takes the smallest colour
  none of its already coloured neighbours holds); the colours take turns 0, 1, ..., C-1,
  0, ...; at its turn every vertex of the colour still below t_end computes
      t_new = min(t_end, Q floor(min(t_plus, tau_v + 1.5 min_w k_vw) / Q - 1e-3))
  and, if t_new > tau_v, emits its tent (ids ascending) with the same layer rule.
A colour class is an independent set, so within a turn no move changes another's target.
The cap on the pole height (1.5 times the vertex's smallest edge step) is a reading: the
paper states no pseudo-time step condition beyond causality, but a vertex that waited
while its neighbours rose would make poles of up to two edge steps, and such tents next to a
material jump made the SAT recursion grow without bound; the cap keeps every pole at most
1.5 edge steps.  The vertex holding the global minimum moves at its colour's turn by at
least its smallest edge step (times quantised), so no C consecutive turns are idle.

Invariant: |tau_v - tau_w| <= k_vw on every edge, hence on every element
grad phi = sum_{j != i} (tau_j - tau_i) grad lambda_j has |grad phi| <= sigma sqrt(eps mu)
(the slope bound 1/(2c) for sigma = 1/2).  The minimum vertex always advances by at least
min k_vw, so the rule never stalls.  Quantising times down to multiples of Q keeps the
invariant and makes two implementations that round differently in the last bits emit
identical tents.

Pins: validate() checks every tent against the definitions (slope bound on every element
after each move, heights positive, element-disjoint patches within a layer, layer order
respects every dependency, flat final front); tests check small cases by hand.
"""
import heapq

import numpy as np

QUANTUM = 2.0 ** -24
SAFETY = 1e-3
POLE_CAP = 1.5     # colour rule: pole height <= POLE_CAP * min_w k_vw


def edge_steps(mesh, sigma, k_elem=None):
    """k_vw per vertex: list of (neighbour ids, k values) aligned with mesh.adj.  k_elem,
    if given, replaces the affine per-element step k_T (curved elements bound the gradient
    of their hat functions over the element, oracle/curved.py)."""
    if k_elem is None:
        norms = np.linalg.norm(mesh.grad_lam, axis=2)              # (ne, d+1)
        sums = norms.sum(axis=1, keepdims=True) - norms             # sum over j != i
        k_T = sigma * np.sqrt(mesh.eps * mesh.mu) / sums.min(axis=1)
    else:
        k_T = np.asarray(k_elem, dtype=np.float64)
    kv = []
    for v in range(mesh.nv):
        nb = mesh.adj[v]
        k = np.full(len(nb), np.inf)
        pos = {int(w): i for i, w in enumerate(nb)}
        for e in mesh.v2e[v]:
            for w in mesh.cells[e]:
                if w != v:
                    i = pos[int(w)]
                    k[i] = min(k[i], k_T[e])
        kv.append(k)
    return kv


def greedy_colouring(mesh):
    """Colour of every vertex: ids ascending, the smallest colour no earlier neighbour holds."""
    colour = -np.ones(mesh.nv, dtype=np.int64)
    for v in range(mesh.nv):
        taken = {int(colour[w]) for w in mesh.adj[v]}
        c = 0
        while c in taken:
            c += 1
        colour[v] = c
    return colour


def pitch(mesh, t_end, sigma=0.5, k_elem=None, rule="min_vertex"):
    """Pitch tents from the flat front 0 to the flat front t_end.

    Returns dict with int arrays vertex, layer and float arrays t_bot, t_top, in
    emission order.  k_elem: per-element steps replacing the affine rule's k_T.
    rule: "min_vertex", "colour" (module docstring) or "auto": both tables, and the one
    whose tents' patch sizes sum to less (the minimum-vertex table on a tie); the returned
    dict then names the chosen rule under "rule"."""
    if rule == "auto":
        a = pitch(mesh, t_end, sigma, k_elem, "min_vertex")
        b = pitch(mesh, t_end, sigma, k_elem, "colour")
        work = lambda t: sum(len(mesh.v2e[int(v)]) for v in t["vertex"])  # noqa: E731
        return {**b, "rule": "colour"} if work(b) < work(a) else {**a, "rule": "min_vertex"}
    if rule == "colour":
        return _pitch_colour(mesh, t_end, sigma, k_elem)
    if rule != "min_vertex":
        raise ValueError(f"unknown pitching rule {rule}")
    nv = mesh.nv
    tau = np.zeros(nv)
    kv = edge_steps(mesh, sigma, k_elem)
    last_layer = -np.ones(nv, dtype=np.int64)
    heap = [(0.0, v) for v in range(nv)]
    heapq.heapify(heap)
    V, TB, TT, L = [], [], [], []
    while heap:
        tv, v = heapq.heappop(heap)
        if tv >= t_end:
            continue
        nb = mesh.adj[v]
        t_plus = np.min(tau[nb] + kv[v])
        t_new = min(t_end, QUANTUM * np.floor(t_plus / QUANTUM - SAFETY))
        if not t_new > tv:
            raise RuntimeError(f"vertex {v} cannot advance")
        lay = 1 + max(last_layer[v], int(np.max(last_layer[nb])))
        last_layer[v] = lay
        V.append(v)
        TB.append(tv)
        TT.append(t_new)
        L.append(lay)
        tau[v] = t_new
        if t_new < t_end:
            heapq.heappush(heap, (t_new, v))
    return {"vertex": np.asarray(V, dtype=np.int64), "t_bot": np.asarray(TB),
            "t_top": np.asarray(TT), "layer": np.asarray(L, dtype=np.int64)}


def _pitch_colour(mesh, t_end, sigma, k_elem):
    tau = np.zeros(mesh.nv)
    kv = edge_steps(mesh, sigma, k_elem)
    cap = np.array([POLE_CAP * np.min(k) for k in kv])
    colour = greedy_colouring(mesh)
    n_colours = int(colour.max()) + 1
    last_layer = -np.ones(mesh.nv, dtype=np.int64)
    V, TB, TT, L = [], [], [], []
    turn, idle = 0, 0
    while np.any(tau < t_end):
        moved = False
        for v in np.nonzero(colour == turn)[0]:
            if tau[v] >= t_end:
                continue
            nb = mesh.adj[v]
            t_plus = min(np.min(tau[nb] + kv[v]), tau[v] + cap[v])
            t_new = min(t_end, QUANTUM * np.floor(t_plus / QUANTUM - SAFETY))
            if t_new > tau[v]:
                lay = 1 + max(last_layer[v], int(np.max(last_layer[nb])))
                last_layer[v] = lay
                V.append(int(v))
                TB.append(tau[v])
                TT.append(t_new)
                L.append(lay)
                tau[v] = t_new
                moved = True
        idle = 0 if moved else idle + 1
        if idle > n_colours:
            raise RuntimeError("colour pitching made no progress")
        turn = (turn + 1) % n_colours
    return {"vertex": np.asarray(V, dtype=np.int64), "t_bot": np.asarray(TB),
            "t_top": np.asarray(TT), "layer": np.asarray(L, dtype=np.int64)}


def validate(mesh, tents, t_end, sigma=0.5, rtol=1e-12):
    """Check a tent list against the definitions; raises AssertionError on violation."""
    s_T = sigma * np.sqrt(mesh.eps * mesh.mu)
    tau = np.zeros(mesh.nv)
    V, TB, TT, L = tents["vertex"], tents["t_bot"], tents["t_top"], tents["layer"]
    # replay in layer order (stable), which must be a valid execution order
    order = np.argsort(L, kind="stable")
    last = -np.ones(mesh.nv, dtype=np.int64)
    for i in order:
        v = int(V[i])
        assert TT[i] > TB[i], f"tent {i}: non-positive height"
        assert tau[v] == TB[i], f"tent {i}: bottom time {TB[i]} != front {tau[v]}"
        tau[v] = TT[i]
        for e in mesh.v2e[v]:
            g = tau[mesh.cells[e]] @ mesh.grad_lam[e]
            assert np.linalg.norm(g) <= s_T[e] * (1 + rtol), f"tent {i}: slope bound on element {e}"
        # layers respect dependencies: previous tents at v or neighbours are in earlier layers
        prev = max(last[v], int(np.max(last[mesh.adj[v]])))
        assert L[i] > prev, f"tent {i}: layer {L[i]} not after a dependency in layer {prev}"
        last[v] = L[i]
    assert np.all(tau == t_end), "final front is not flat at t_end"
    for lay in np.unique(L):
        els = np.concatenate([mesh.v2e[int(v)] for v in V[L == lay]])
        assert len(els) == len(np.unique(els)), f"layer {lay}: patches overlap"
    return True

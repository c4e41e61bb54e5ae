"""Exact and by-definition references for tiny graphs (test code only).

These compute the expected spread I(S) straight from the diffusion models of
Section 2.1, independently of RR sets:
  * IC: enumerate all 2^m live-edge graphs (edge live with probability w),
    spread = expected number of nodes reachable from S;
  * LT: enumerate every choice of at most one live in-edge per node (edge i
    of v with probability w_i, none with 1 - sum w) -- Kempe, Kleinberg,
    Tardos (KDD 2003) prove this equals the threshold model -- and, as a
    check of that reading, simulate the threshold model itself (lambda_v
    uniform, activate when the active in-weight reaches lambda_v).
They share nothing with the oracle.
"""
from __future__ import annotations

import itertools
from collections import defaultdict

import numpy as np


def _reach(n, live_edges, S, node_w=None):
    """Nodes reachable from S over live edges: their number, or the sum of
    their weights node_w[v] (the targeted spread of Section 7.3)."""
    out = defaultdict(list)
    for u, v in live_edges:
        out[u].append(v)
    seen = set(S)
    stack = list(S)
    while stack:
        u = stack.pop()
        for v in out[u]:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    if node_w is None:
        return len(seen)
    return float(sum(node_w[v] for v in seen))


def ic_exact_spread(n, edges, S, node_w=None):
    """edges: list of (u, v, p). Exact I(S) under IC by enumeration (with
    node_w: the expected total weight of the reached nodes)."""
    m = len(edges)
    total = 0.0
    for mask in range(1 << m):
        prob = 1.0
        live = []
        for i, (u, v, p) in enumerate(edges):
            if mask >> i & 1:
                prob *= p
                live.append((u, v))
            else:
                prob *= 1.0 - p
        if prob == 0.0:
            continue
        total += prob * _reach(n, live, S, node_w)
    return total


def lt_exact_spread(n, edges, S, node_w=None):
    """edges: list of (u, v, w) with sum of w into each v <= 1. Exact I(S)
    (with node_w: the expected total weight of the reached nodes)."""
    into = defaultdict(list)
    for u, v, w in edges:
        into[v].append((u, w))
    nodes = list(range(n))
    choices = []
    for v in nodes:
        opts = [(None, 1.0 - sum(w for _, w in into[v]))] + [(u, w) for u, w in into[v]]
        choices.append(opts)
    total = 0.0
    for combo in itertools.product(*choices):
        prob = 1.0
        live = []
        for v, (u, w) in zip(nodes, combo):
            prob *= w
            if u is not None:
                live.append((u, v))
        if prob <= 0.0:
            continue
        total += prob * _reach(n, live, S, node_w)
    return total


def lt_threshold_mc(n, edges, S, trials, seed=0):
    """Monte Carlo of the LT model as defined (random thresholds)."""
    rng = np.random.default_rng(seed)
    into = defaultdict(list)
    for u, v, w in edges:
        into[v].append((u, w))
    acc = 0
    for _ in range(trials):
        lam = rng.random(n)
        active = set(S)
        changed = True
        while changed:
            changed = False
            for v in range(n):
                if v in active:
                    continue
                if sum(w for u, w in into[v] if u in active) >= lam[v]:
                    active.add(v)
                    changed = True
        acc += len(active)
    return acc / trials


def ic_forward_mc(n, edges, S, trials, seed=0):
    """Monte Carlo of the IC cascade as defined (each newly active node gets
    one chance per out-edge)."""
    rng = np.random.default_rng(seed)
    out = defaultdict(list)
    for u, v, p in edges:
        out[u].append((v, p))
    acc = 0
    for _ in range(trials):
        active = set(S)
        frontier = list(S)
        while frontier:
            nxt = []
            for u in frontier:
                for v, p in out[u]:
                    if v not in active and rng.random() < p:
                        active.add(v)
                        nxt.append(v)
            frontier = nxt
        acc += len(active)
    return acc / trials


def exact_opt(n, k, spread):
    """Exhaustive best size-k set under `spread(S)`."""
    best, best_s = -1.0, None
    for S in itertools.combinations(range(n), k):
        val = spread(S)
        if val > best + 1e-12:
            best, best_s = val, S
    return best_s, best


def random_tiny_graph(rng, n, m, model):
    """Random digraph without self-loops or repeated pairs; IC probabilities
    uniform in [0.05, 0.95]; LT weights with sum <= 1 per node."""
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    idx = rng.choice(len(pairs), size=m, replace=False)
    chosen = sorted((pairs[i] for i in idx), key=lambda e: (e[1], e[0]))
    edges = []
    if model == 0:
        for u, v in chosen:
            edges.append((u, v, float(np.float32(rng.uniform(0.05, 0.95)))))
    else:
        by_v = defaultdict(list)
        for u, v in chosen:
            by_v[v].append(u)
        for v in sorted(by_v):
            raw = rng.uniform(0.1, 1.0, size=len(by_v[v]))
            scale = rng.uniform(0.5, 1.0) / raw.sum()
            for u, r in zip(by_v[v], raw):
                w = np.float32(r * scale)
                edges.append((u, v, float(w)))
    return edges


def arrays(edges):
    src = np.array([e[0] for e in edges], dtype=np.uint32)
    dst = np.array([e[1] for e in edges], dtype=np.uint32)
    w = np.array([e[2] for e in edges], dtype=np.float32)
    return src, dst, w

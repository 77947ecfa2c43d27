"""Contraction path, contraction tree, cost formulas, lifetimes, Algorithm 1.

Written from the paper:

* contraction tree B (Sec. 2.1.1): one node per contraction, its tensor's
  indices are the symmetric difference of its children's (Lemma 1);
* Eq. (1)  C(B)   = sum over contractions of 2^|s_v1 u s_v2 u s_v3|;
  read here as the contraction (internal) nodes only; leaf reads and the
  final scalar node carry no multiply-adds;
* Eq. (2)  O(B,S) = C_slice(B) 2^|S| / C_original(B);
* Eq. (4)  C(B,S) = sum_V 2^(|s_V| + |S| - |S n s_V|);
* space cost = largest tensor, max 2^rank;
* lifetime of an index (Sec. 3.1 Definition) = the tree tensors holding it;
* stem (Sec. 4.2) = the most computationally intensive root-to-leaf path;
* Algorithm 1 (slice finder) on the stem, then a fix-up for off-stem tensors.

The greedy path is not in the paper (which takes its paths from cotengra);
it follows the usual greedy rule: among tensor pairs sharing an index,
contract the pair minimising size(out) - alpha (size(a) + size(b)),
optionally scaled by (1 +- tau u) with a keyed uniform u (randomised
greedy); ties go to the lexicographically smallest (lower id, higher id);
when no pair shares an index, the two lowest ids are joined by an outer
product. SSA ids: leaves 0..L-1, the k-th contraction creates L+k.

Readings of the slice finder (Sec. 4.2, Algorithm 1; the paper does not
give tie-breaks):
* ranks are taken after removing the indices already in S; the stem
  tensors at or below t are set aside before each choice, so the two ends
  compared are those of the over-cap part (the stem always starts at a
  leaf; whenever that leaf fits, this is the order of the paper's loop);
* of the two ends the one of smaller rank is fixed next, the root-side one
  on a tie;
* "longest lifetime" = the index's stem lifetime (an interval of stem
  positions) covers the most over-cap stem tensors, then the most tensors
  of the whole tree hold it, then the smaller index id;
* off-stem tensors still above t afterwards (SSA order): add their unsliced
  index with the longest whole-tree lifetime (then smaller id) until they
  fit.

Slice refiner (Sec. 4.3, Algorithms 2-4), readings where the paper is
silent:
* lifetime of an index = every tree tensor holding it (leaves included);
  ``dim`` = rank after removing the current S; critical tensors of a sliced
  index = tensors of its lifetime whose dim equals t (Algorithm 3);
* candidates = the unsliced indices whose lifetime contains all of its
  critical tensors (Sec. 4.3; the same set as Algorithm 4's intersection of
  the critical tensors' index sets), in ascending id;
* a sliced index whose lifetime holds no critical tensor is dropped from S
  (it reduces no tensor to the cap, Sec. 4.3), which lowers C(B,S);
* candidate moves act on the chosen slot in turn: each proposal replaces
  the slot's current occupant, so the cap is kept by construction;
* T starts at t0 and is multiplied by alpha after every ``iters_per_temp``
  iterations; the loop runs until T < tf (at least once); acceptance of a
  costlier set: keyed uniform < exp((C_ori - C_new) / C_ori / T), with the
  two big integers rounded to doubles; the best set seen is returned;
* the first ``n_fixed`` entries of S (pre-sliced indices) are never moved.
* random draws: iteration i picks slot n_fixed + floor(u (|S| - n_fixed))
  with u = keyed_uniform(seed, i, 0, 0); candidate c is accepted uphill
  when keyed_uniform(seed, i, 1, c) < p.

Subtree reconfiguration (a path improvement in the spirit of the local
tuning of the contraction tree cited in Sec. 2.1.2; the paper takes its
paths from cotengra instead): for every contraction node v in SSA order,
grow a frontier from v by repeatedly replacing the frontier node with the
largest node set (after removing S; ties: smaller id) by its two children,
up to k tensors; re-contract the frontier in the order of least summed node
cost 2^|s_v - S| (exhaustive over subsets; with a target t, intermediate
tensors above t after S are not allowed); keep the new subtree when it is
strictly cheaper. Costs saturate at 2^120 (no finite tree reaches it).
Ties in the subset search keep the first minimum when the split's smaller
part (as a bit mask over the frontier) runs downward. New nodes reuse the
subtree's ids; after every sweep the tree is written out again as an SSA
path in post order (left child first).

Greedy-overhead slicer (the strategy attributed to cotengra in Sec. 2.1.2):
while some tensor is above t, slice the index, among those of tensors above
t, whose addition gives the smallest C(B,S); ties: held by the most
tensors above t, then the smaller id.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple


MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 (Steele, Lea, Flood 2014): one step from state x."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def keyed_uniform(seed: int, step: int, a: int, b: int) -> float:
    """Uniform double in [0, 1) that depends only on (seed, step, a, b)."""
    h = splitmix64(seed & MASK64)
    h = splitmix64(h ^ step)
    h = splitmix64(h ^ a)
    h = splitmix64(h ^ b)
    return (h >> 11) * (2.0 ** -53)


def pair_key(rc: int, ra: int, rb: int, alpha: float, tau: float, u: float) -> float:
    """Greedy score of contracting two tensors of ranks ra, rb into rank rc,
    in IEEE double, in this exact order of operations."""
    t1 = math.ldexp(1.0, ra) + math.ldexp(1.0, rb)
    t2 = alpha * t1
    base = math.ldexp(1.0, rc) - t2
    if tau > 0.0:
        f = tau * u
        if base > 0.0:
            base = base * (1.0 + f)
        else:
            base = base * (1.0 - f)
    return base


def greedy_path(leaf_indices: Sequence[Sequence[int]], alpha: float = 1.0, tau: float = 0.0,
                seed: int = 0, exclude: Sequence[int] = ()) -> List[Tuple[int, int]]:
    """Greedy SSA path; alpha = 1, tau = 0 is the plain rule, other values
    give the randomised variant (key in ``pair_key``, noise from
    ``keyed_uniform``). Indices in ``exclude`` are ignored."""
    ex = set(exclude)
    L = len(leaf_indices)
    live: Dict[int, frozenset] = {i: frozenset(x for x in ix if x not in ex)
                                  for i, ix in enumerate(leaf_indices)}
    owner: Dict[int, set] = {}
    for t, ix in live.items():
        for x in ix:
            owner.setdefault(x, set()).add(t)
    path = []
    nxt = L
    step = 0
    while len(live) > 1:
        best = None
        for x, ts in owner.items():
            if len(ts) != 2:
                continue
            a, b = sorted(ts)
            ia, ib = live[a], live[b]
            u = keyed_uniform(seed, step, a, b) if tau > 0.0 else 0.0
            key = (pair_key(len(ia ^ ib), len(ia), len(ib), alpha, tau, u), a, b)
            if best is None or key < best:
                best = key
        if best is None:
            a, b = sorted(live)[:2]
        else:
            _, a, b = best
        new = live[a] ^ live[b]
        for x in live[a] | live[b]:
            owner[x].discard(a)
            owner[x].discard(b)
            if x in new:
                owner[x].add(nxt)
            elif not owner[x]:
                del owner[x]
        del live[a], live[b]
        live[nxt] = new
        path.append((a, b))
        nxt += 1
        step += 1
    return path


class Tree:
    """Rooted binary contraction tree of an SSA path."""

    def __init__(self, leaf_indices: Sequence[Sequence[int]], path: Sequence[Tuple[int, int]]):
        self.L = len(leaf_indices)
        self.path = [tuple(p) for p in path]
        self.sets: List[frozenset] = [frozenset(ix) for ix in leaf_indices]
        self.children: List[Optional[Tuple[int, int]]] = [None] * self.L
        self.parent: List[int] = [-1] * (self.L + len(self.path))
        for k, (a, b) in enumerate(self.path):
            v = self.L + k
            self.sets.append(self.sets[a] ^ self.sets[b])
            self.children.append((a, b))
            self.parent[a] = v
            self.parent[b] = v
        self.root = len(self.sets) - 1

    def nodes(self) -> range:
        return range(self.L, len(self.sets))

    def node_set(self, v: int) -> frozenset:
        """s_v1 u s_v2 u s_v3 of contraction node v."""
        a, b = self.children[v]
        return self.sets[a] | self.sets[b]

    def cost(self) -> int:
        """Eq. (1)."""
        return sum(1 << len(self.node_set(v)) for v in self.nodes())

    def sliced_cost(self, S: Sequence[int]) -> int:
        """Eq. (4)."""
        S = set(S)
        tot = 0
        for v in self.nodes():
            sv = self.node_set(v)
            tot += 1 << (len(sv) + len(S) - len(S & sv))
        return tot

    def overhead(self, S: Sequence[int]) -> float:
        """Eq. (2)."""
        return self.sliced_cost(S) / self.cost()

    def space(self, S: Sequence[int] = ()) -> int:
        S = set(S)
        return max(1 << len(s - S) for s in self.sets)

    def lifetime(self, index: int) -> List[int]:
        """Tree tensors (node ids) holding ``index``."""
        return [v for v, s in enumerate(self.sets) if index in s]

    def stem(self) -> List[int]:
        """Root-to-leaf path of largest summed node cost, as node ids
        ordered leaf -> root. Ties: the child with the larger subtree cost,
        then the smaller id."""
        best: Dict[int, int] = {}
        sub: Dict[int, int] = {}
        for v in range(len(self.sets)):
            if v < self.L:
                best[v] = 0
                sub[v] = 0
            else:
                a, b = self.children[v]
                c = 1 << len(self.node_set(v))
                best[v] = c + max(best[a], best[b])
                sub[v] = c + sub[a] + sub[b]
        out = [self.root]
        v = self.root
        while v >= self.L:
            a, b = self.children[v]
            v = min((a, b), key=lambda u: (-best[u], -sub[u], u))
            out.append(v)
        return out[::-1]


def stem_intervals(tree: Tree, stem: Sequence[int]) -> Dict[int, Tuple[int, int]]:
    """Lifetime of every index on the stem, as a closed interval of stem
    positions. By the Linearity theorem (supplement) the tensors holding an
    index lie on one path of the tree, and a path meets the stem (another
    path) in one contiguous stretch, so an interval describes it exactly."""
    iv: Dict[int, Tuple[int, int]] = {}
    for p, v in enumerate(stem):
        for x in tree.sets[v]:
            lo, _ = iv.get(x, (p, p))
            iv[x] = (lo, p)
    return iv


def pick_end(over: Sequence[int], rank) -> int:
    """Which end of the over-cap part of the stem is fixed next (Sec. 4.2:
    the search starts from both ends of the stem): the end tensor of smaller
    rank, the root-side end when the two are equal. ``over`` holds stem
    positions, leaf side first; ``rank(p)`` is the rank after slicing."""
    return over[0] if rank(over[0]) < rank(over[-1]) else over[-1]


def lifetime_order(cands: Sequence[int], span: Dict[int, int], whole: Dict[int, int]) -> List[int]:
    """Indices ordered best first for slicing (Sec. 4.2: an index whose
    lifetime covers more of the remaining over-cap stem is preferred):
    longer span over the over-cap stem tensors, then more tree tensors
    holding the index, then the smaller id."""
    return sorted(cands, key=lambda x: (-span[x], -whole[x], x))


def slice_finder(tree: Tree, t: int, pre: Sequence[int] = ()) -> List[int]:
    """Lifetime-based slice finder (Sec. 4.2, Algorithm 1) on the stem,
    then the off-stem fix-up, starting from the already-sliced indices
    ``pre``. Returns S = pre + the indices in the order they were added
    (bit j of a slice id is the value of S[j]). t < 0 means no cap.

    The stem tensors whose rank after slicing exceeds t form the part of
    the stem still to fix. Each round takes one end of that part (the M_1
    of the paper; the rest is M_2), slices as many of its unsliced indices
    as it exceeds t by, choosing those whose stem lifetime covers most of
    the over-cap tensors, and drops the tensors that now fit. Tensors off
    the stem that still exceed t (the paper says most branches fit, not
    all) are fixed afterwards in id order, each by its unsliced index held
    by the most tree tensors (then the smaller id)."""
    S: List[int] = list(pre)
    if t < 0:
        return S
    if pre:
        # the pre-sliced indices are fixed before anything else: the tree,
        # its stem and all lifetimes are taken without them
        ps = set(pre)
        tree = Tree([[x for x in tree.sets[v] if x not in ps] for v in range(tree.L)], tree.path)
    inS = set()

    def rank(v):
        return len(tree.sets[v] - inS)

    stem = tree.stem()
    iv = stem_intervals(tree, stem)
    whole: Dict[int, int] = {}
    for s in tree.sets:
        for x in s:
            whole[x] = whole.get(x, 0) + 1
    over = [p for p, v in enumerate(stem) if rank(v) > t]
    while over:
        p = pick_end(over, lambda q: rank(stem[q]))
        v = stem[p]
        cands = [x for x in tree.sets[v] if x not in inS]
        span = {x: sum(1 for q in over if iv[x][0] <= q <= iv[x][1]) for x in cands}
        for x in lifetime_order(cands, span, whole)[:rank(v) - t]:
            S.append(x)
            inS.add(x)
        over = [q for q in over if rank(stem[q]) > t]
    for v in range(len(tree.sets)):
        while rank(v) > t:
            x = min((y for y in tree.sets[v] if y not in inS), key=lambda y: (-whole[y], y))
            S.append(x)
            inS.add(x)
    return S


def path_search(leaf_indices, t: int, pre: Sequence[int] = (), alphas=(1.0,), taus=(0.0,),
                n_seeds: int = 1, seed_base: int = 0, reconf_k: int = 0, reconf_sweeps: int = 4):
    """Randomised greedy trials (alpha-major, then tau, then seed; tau = 0
    runs seed 0 only), each followed by the slice finder; keep the smallest
    (C(B,S), |S|, trial number). Returns (path, S, trial). With reconf_k >= 3
    each trial's path goes through ``reconfigure`` before the slice finder
    (S = pre, no cap) and after it (the trial's S, cap t)."""
    best = None
    trial = 0
    for alpha in alphas:
        for tau in taus:
            for sd in range(n_seeds if tau > 0.0 else 1):
                p = greedy_path(leaf_indices, alpha, tau, seed_base + sd, exclude=pre)
                if reconf_k >= 3:
                    p = reconfigure(leaf_indices, p, reconf_k, reconf_sweeps, pre, -1)
                tr = Tree(leaf_indices, p)
                S = slice_finder(tr, t, pre)
                if reconf_k >= 3 and t >= 0:
                    p = reconfigure(leaf_indices, p, reconf_k, reconf_sweeps, S, t)
                    tr = Tree(leaf_indices, p)
                key = (tr.sliced_cost(S), len(S), trial)
                if best is None or key < best[0]:
                    best = (key, p, S, trial)
                trial += 1
    return best[1], best[2], best[3]


def critical_tensors(tree: Tree, S: Sequence[int], index: int, t: int) -> List[int]:
    """The critical tensors of a sliced index (Sec. 4.3; Algorithm 3): the
    tensors of its lifetime whose rank after slicing S is exactly t."""
    Sset = set(S)
    return [v for v in tree.lifetime(index) if len(tree.sets[v] - Sset) == t]


def candidate_indices(tree: Tree, crit: Sequence[int], S: Sequence[int]) -> List[int]:
    """Replacements for a sliced index with critical tensors ``crit``
    (Sec. 4.3; Algorithm 4): the unsliced indices whose lifetime contains
    every critical tensor, ascending id. Slicing one of them instead keeps
    every critical tensor at t, so the cap still holds."""
    need = set(crit)
    Sset = set(S)
    everywhere = set().union(*(tree.sets[v] for v in crit))
    return sorted(x for x in everywhere if x not in Sset and need <= set(tree.lifetime(x)))


def fits(tree: Tree, S: Sequence[int], t: int) -> bool:
    Sset = set(S)
    return all(len(s - Sset) <= t for s in tree.sets)


def slice_refine(tree: Tree, t: int, S: Sequence[int], n_fixed: int = 0, t0: float = 1.0,
                 alpha: float = 0.98, tf: float = 1e-3, iters_per_temp: int = 1,
                 seed: int = 0) -> Tuple[List[int], dict]:
    """Algorithm 2 (simulated annealing over edge replacements). Returns the
    best slicing set seen and counters (iterations, proposals, accepted,
    dropped)."""
    if not fits(tree, S, t):
        raise ValueError("the input slicing set does not meet the cap")
    cur = list(S)
    cur_c = tree.sliced_cost(cur)
    best, best_c = list(cur), cur_c
    stats = {"iterations": 0, "proposals": 0, "accepted": 0, "dropped": 0}
    T = t0
    it = 0
    while True:
        for _ in range(iters_per_temp):
            free = len(cur) - n_fixed
            if free <= 0:
                break
            u = keyed_uniform(seed, it, 0, 0)
            slot = n_fixed + min(int(u * free), free - 1)
            crit = critical_tensors(tree, cur, cur[slot], t)
            if not crit:
                del cur[slot]
                cur_c = tree.sliced_cost(cur)
                stats["dropped"] += 1
            else:
                for c in candidate_indices(tree, crit, cur):
                    prop = list(cur)
                    prop[slot] = c
                    new_c = tree.sliced_cost(prop)
                    stats["proposals"] += 1
                    if new_c < cur_c:
                        take = True
                    else:
                        p = math.exp(-(float(new_c - cur_c) / float(cur_c)) / T)
                        take = keyed_uniform(seed, it, 1, c) < p
                    if take:
                        cur, cur_c = prop, new_c
                        stats["accepted"] += 1
                    if cur_c < best_c:
                        best, best_c = list(cur), cur_c
            if cur_c < best_c:
                best, best_c = list(cur), cur_c
            it += 1
        stats["iterations"] = it
        T = T * alpha
        if T < tf or len(cur) <= n_fixed:
            break
    return best, stats


def greedy_overhead_slicer(tree: Tree, t: int, pre: Sequence[int] = ()) -> List[int]:
    """Greedy slicing by least overhead: add, one at a time, the index that
    gives the smallest C(B,S) among the unsliced indices of tensors above t
    (ties: most tensors above t holding it, then smaller id)."""
    S = list(pre)
    if t < 0:
        return S
    while True:
        Sset = set(S)
        big = [v for v, s in enumerate(tree.sets) if len(s - Sset) > t]
        if not big:
            return S
        count: Dict[int, int] = {}
        for v in big:
            for x in tree.sets[v] - Sset:
                count[x] = count.get(x, 0) + 1
        pick = min(count, key=lambda x: (tree.sliced_cost(S + [x]), -count[x], x))
        S.append(pick)


SAT = 1 << 120


def _sat(x: int) -> int:
    return x if x < SAT else SAT


def reconfigure(leaf_indices: Sequence[Sequence[int]], path: Sequence[Tuple[int, int]], k: int,
                sweeps: int = 1, S: Sequence[int] = (), t: int = -1) -> List[Tuple[int, int]]:
    """Subtree reconfiguration; returns the new SSA path (same leaves)."""
    Sset = frozenset(S)
    L = len(leaf_indices)
    sets: List[frozenset] = [frozenset(ix) for ix in leaf_indices]
    kids: List[Optional[Tuple[int, int]]] = [None] * L
    for a, b in path:
        sets.append(sets[a] ^ sets[b])
        kids.append((a, b))
    n = len(sets)

    def node_cost(sa, sb):
        return _sat(1 << len((sa | sb) - Sset)) if len((sa | sb) - Sset) < 120 else SAT

    for _ in range(sweeps):
        improved = False
        for v in range(L, n):
            front = [v]
            while len(front) < k:
                inner = [u for u in front if kids[u] is not None]
                if not inner:
                    break
                u = max(inner, key=lambda u: (len((sets[kids[u][0]] | sets[kids[u][1]]) - Sset), -u))
                front.remove(u)
                front.extend(kids[u])
            m = len(front)
            if m < 3:
                continue
            inner_nodes: List[int] = []

            def collect(u):
                if u in front:
                    return
                inner_nodes.append(u)
                collect(kids[u][0])
                collect(kids[u][1])

            collect(v)
            old = 0
            for u in inner_nodes:
                old = _sat(old + node_cost(sets[kids[u][0]], sets[kids[u][1]]))
            if old >= SAT:
                continue
            # exhaustive search over subsets of the frontier
            tens = [frozenset()] * (1 << m)
            for M in range(1, 1 << m):
                low = M & -M
                tens[M] = tens[M ^ low] ^ sets[front[low.bit_length() - 1]]
            best = [0] * (1 << m)
            choice = [0] * (1 << m)
            full = (1 << m) - 1
            for M in range(1, 1 << m):
                if M & (M - 1) == 0:
                    continue
                if t >= 0 and M != full and len(tens[M] - Sset) > t:
                    best[M] = SAT
                    continue
                bc, bsub = None, 0
                sub = (M - 1) & M
                while sub:
                    o = M ^ sub
                    if sub < o:
                        c = _sat(_sat(best[sub] + best[o]) + node_cost(tens[sub], tens[o]))
                        if bc is None or c < bc:
                            bc, bsub = c, sub
                    sub = (sub - 1) & M
                best[M] = bc
                choice[M] = bsub
            if best[full] >= old:
                continue
            improved = True

            def nest(M):
                if M & (M - 1) == 0:
                    return front[M.bit_length() - 1]
                return (nest(choice[M]), nest(M ^ choice[M]))

            pool = [u for u in inner_nodes if u != v]

            def assign(tr, is_root):
                if not isinstance(tr, tuple):
                    return tr
                a = assign(tr[0], False)
                b = assign(tr[1], False)
                u = v if is_root else pool.pop()
                kids[u] = (a, b)
                sets[u] = sets[a] ^ sets[b]
                return u

            assign(nest(full), True)
        # write the tree out again in post order
        order: List[int] = []
        stack = [(n - 1, False)]
        while stack:
            u, done = stack.pop()
            if kids[u] is None:
                continue
            if done:
                order.append(u)
            else:
                stack.append((u, True))
                stack.append((kids[u][1], False))
                stack.append((kids[u][0], False))
        newid = list(range(L)) + [0] * (n - L)
        new_path = []
        for u in order:
            a, b = kids[u]
            newid[u] = L + len(new_path)
            new_path.append((newid[a], newid[b]))
        sets = sets[:L]
        kids = kids[:L]
        for a, b in new_path:
            sets.append(sets[a] ^ sets[b])
            kids.append((a, b))
        if not improved:
            break
    return [kids[u] for u in range(L, n)]

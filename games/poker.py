"""Multi-round private-rank poker, generated per deal from one betting template.

This is the family of the large synthetic workloads: one chance node deals
each player a distinct private rank; up to three betting rounds follow, with a
chance node revealing one public card between rounds. Actions are fold (only
when facing a bet), call (check when not facing), pot-raise (call, then raise
by the pot after calling) and all-in; both raise kinds count toward the cap of
raises per round; a pot-raise is legal only if it commits strictly less than
the stack; nobody raises over an all-in; a called all-in goes straight to a
showdown terminal. Ante 1. Showdown: the higher private rank wins the
opponent's commitment (ranks are distinct, so there are no ties).

The betting skeleton of one deal does not depend on the cards, so it is built
once as a template (Python) and replicated over all deals with numpy. An
infoset is (player, own rank, public cards by identity, betting history).

``subgame`` builds the batched-solving family: the game starts at a later
round with a given pot and board, root beliefs drawn from Dirichlet(1) over
private ranks, and payoffs divided by the largest absolute payoff.
"""
from __future__ import annotations

import math

import numpy as np

from .tuple import Game

KIND_CHANCE, KIND_P1, KIND_P2, KIND_TERM = 0, 1, 2, 3
TERM_FOLD1, TERM_FOLD2, TERM_SHOW = 0, 1, 2


class _Template:
    """Betting/chance skeleton below one deal (no card identities)."""

    def __init__(self, n_rounds: int, fanouts, cap: int, stack: int, c0: int):
        self.parent: list[int] = []
        self.action: list[int] = []
        self.kind: list[int] = []
        self.nact: list[int] = []
        self.bet: list[int] = []       # betting-history id (decision nodes)
        self.slot: list[tuple] = []    # public card indices dealt inside this subgame
        self.term: list[int] = []
        self.commit: list[int] = []
        self.depth: list[int] = []
        self.info: list[tuple] = []    # decision nodes: (c1, c2, raises, last, round, amask)
        self._bet_ids: dict = {}
        self.n_rounds, self.fanouts, self.cap, self.stack = n_rounds, list(fanouts), cap, stack
        self._round(-1, -1, 0, c0, c0, 0, 1, False, (), (), 0)

    def _new(self, parent, action, kind, nact, bet, slot, depth, term=-1, commit=0, info=None):
        self.parent.append(parent); self.action.append(action); self.kind.append(kind)
        self.nact.append(nact); self.bet.append(bet); self.slot.append(slot)
        self.term.append(term); self.commit.append(commit); self.depth.append(depth)
        self.info.append(info if info is not None else (0, 0, 0, 0, 0, 0))
        return len(self.parent) - 1

    def _bet_id(self, path):
        i = self._bet_ids.get(path)
        if i is None:
            i = len(self._bet_ids)
            self._bet_ids[path] = i
        return i

    def _round(self, parent, action, rnd, c1, c2, raises, actor, facing, path, slot, depth):
        me, op = (c1, c2) if actor == 1 else (c2, c1)
        acts = []
        if facing:
            acts.append(("f",))
        acts.append(("c",))
        if raises < self.cap and op < self.stack:
            pot = c1 + c2 + (op - me)
            if op + pot < self.stack:
                acts.append(("p", op + pot))
            if me < self.stack:
                acts.append(("a", self.stack))
        kind = KIND_P1 if actor == 1 else KIND_P2
        this_round = path[len(path) - path[::-1].index("|"):] if "|" in path else path
        last = {"c": 1, "p": 2, "a": 3}.get(this_round[-1], 0) if this_round else 0
        amask = sum({"f": 1, "c": 2, "p": 4, "a": 8}[a[0]] for a in acts)
        v = self._new(parent, action, kind, len(acts), self._bet_id(path), slot, depth,
                      info=(c1, c2, raises, last, rnd, amask))
        for a, act in enumerate(acts):
            if act[0] == "f":
                self._new(v, a, KIND_TERM, 0, -1, slot, depth + 1,
                          TERM_FOLD1 if actor == 1 else TERM_FOLD2, me)
            elif act[0] == "c":
                m = max(c1, c2)
                if facing or actor == 2:
                    if m >= self.stack or rnd == self.n_rounds - 1:
                        self._new(v, a, KIND_TERM, 0, -1, slot, depth + 1, TERM_SHOW, m)
                    else:
                        self._chance(v, a, rnd + 1, m, path + ("c", "|"), slot, depth + 1)
                else:
                    self._round(v, a, rnd, c1, c2, raises, 2, False, path + ("c",), slot, depth + 1)
            else:
                n1, n2 = (act[1], c2) if actor == 1 else (c1, act[1])
                self._round(v, a, rnd, n1, n2, raises + 1, 3 - actor, True, path + (act[0],),
                            slot, depth + 1)

    def _chance(self, parent, action, rnd, c, path, slot, depth):
        f = self.fanouts[rnd - 1]
        v = self._new(parent, action, KIND_CHANCE, f, -1, slot, depth)
        for i in range(f):
            self._round(v, i, rnd, c, c, 0, 1, False, path, slot + (i,), depth + 1)


def _arrays(t: _Template) -> dict:
    n = len(t.parent)
    slots = np.full((n, 2), -1, dtype=np.int64)
    for i, s in enumerate(t.slot):
        for j, x in enumerate(s):
            slots[i, j] = x
    return {
        "parent": np.asarray(t.parent, dtype=np.int64),
        "action": np.asarray(t.action, dtype=np.int64),
        "kind": np.asarray(t.kind, dtype=np.int64),
        "nact": np.asarray(t.nact, dtype=np.int64),
        "bet": np.asarray(t.bet, dtype=np.int64),
        "slot": slots,
        "term": np.asarray(t.term, dtype=np.int64),
        "commit": np.asarray(t.commit, dtype=np.int64),
        "info": np.asarray(t.info, dtype=np.int64),
        "depth": np.asarray(t.depth, dtype=np.int64),
        "n": n,
    }


def template_size(n_ranks: int, n_rounds: int, cap: int, stack: int, c0: int = 1,
                  board_size: int = 0) -> int:
    """Node count below one deal (memoised recursion; no template is built)."""
    fan = [n_ranks - 2 - board_size - k for k in range(n_rounds - 1)]
    memo: dict = {}

    def rnd(r, c1, c2, raises, actor, facing):
        key = (r, c1, c2, raises, actor, facing)
        if key in memo:
            return memo[key]
        me, op = (c1, c2) if actor == 1 else (c2, c1)
        total = 1
        if facing:
            total += 1
        m = max(c1, c2)
        if facing or actor == 2:
            total += 1 if (m >= stack or r == n_rounds - 1) else 1 + fan[r] * rnd(r + 1, m, m, 0, 1, False)
        else:
            total += rnd(r, c1, c2, raises, 2, False)
        if raises < cap and op < stack:
            pot = c1 + c2 + (op - me)
            if op + pot < stack:
                n1, n2 = (op + pot, c2) if actor == 1 else (c1, op + pot)
                total += rnd(r, n1, n2, raises + 1, 3 - actor, True)
            if me < stack:
                n1, n2 = (stack, c2) if actor == 1 else (c1, stack)
                total += rnd(r, n1, n2, raises + 1, 3 - actor, True)
        memo[key] = total
        return total

    return rnd(0, c0, c0, 0, 1, False)


def poker_game(n_ranks: int = 13, n_rounds: int = 3, cap: int = 3, stack: int = 400,
               c0: int = 1, board=(), deal_prob=None, scale: bool = False,
               name: str | None = None, max_deals: int | None = None) -> Game:
    """Build the game. ``deal_prob`` (optional) maps the ordered deal list to
    probabilities; ``board`` holds public cards already dealt before the game.
    ``max_deals`` keeps only the first deals (a bounded sample of the same game, with the
    root's probabilities renormalised over the kept deals)."""
    board = tuple(int(x) for x in board)
    free = [r for r in range(n_ranks) if r not in board]
    deals = np.asarray([(a, b) for a in free for b in free if a != b], dtype=np.int64)
    if max_deals is not None:
        deals = deals[:max_deals]
        if deal_prob is not None:
            deal_prob = np.asarray(deal_prob, dtype=np.float64)[:max_deals]
            deal_prob = deal_prob / deal_prob.sum()
    nd = len(deals)
    fan = [n_ranks - 2 - len(board) - k for k in range(n_rounds - 1)]
    tpl = _arrays(_Template(n_rounds, fan, cap, stack, c0))
    tn = tpl["n"]

    # remaining-card tables: pub1[d, i] and pub2[d, i, j] (card identities)
    pub1 = np.full((nd, max(fan[0] if fan else 1, 1)), -1, dtype=np.int64)
    pub2 = np.full((nd, max(fan[0] if fan else 1, 1), max(fan[1] if len(fan) > 1 else 1, 1)), -1,
                   dtype=np.int64)
    for d, (r1, r2) in enumerate(deals):
        rest = [r for r in free if r != r1 and r != r2]
        if fan:
            for i in range(fan[0]):
                pub1[d, i] = rest[i]
                if len(fan) > 1:
                    rest2 = [r for r in rest if r != rest[i]]
                    for j in range(fan[1]):
                        pub2[d, i, j] = rest2[j]

    n = 1 + nd * tn
    parent = np.empty(n, dtype=np.int64)
    action = np.empty(n, dtype=np.int64)
    parent[0] = -1
    action[0] = -1
    d_idx = np.repeat(np.arange(nd, dtype=np.int64), tn)
    t_idx = np.tile(np.arange(tn, dtype=np.int64), nd)
    base = 1 + d_idx * tn
    tpar = tpl["parent"][t_idx]
    parent[1:] = np.where(tpar < 0, 0, base + tpar)
    action[1:] = np.where(tpar < 0, d_idx, tpl["action"][t_idx])
    kind = tpl["kind"][t_idx]
    del tpar

    r1 = deals[d_idx, 0]
    r2 = deals[d_idx, 1]
    s1 = tpl["slot"][t_idx, 0]
    s2 = tpl["slot"][t_idx, 1]
    p1 = np.where(s1 >= 0, pub1[d_idx, np.maximum(s1, 0)], -1)
    p2 = np.where(s2 >= 0, pub2[d_idx, np.maximum(s1, 0), np.maximum(s2, 0)], -1)
    del s1, s2

    node_infoset = np.full(n, -1, dtype=np.int64)
    # player infosets: (betting history, public cards, own rank, player)
    dec = np.flatnonzero((kind == KIND_P1) | (kind == KIND_P2))
    own = np.where(kind[dec] == KIND_P1, r1[dec], r2[dec])
    R1 = n_ranks + 1
    key = ((((tpl["bet"][t_idx[dec]] * R1 + (p1[dec] + 1)) * R1 + (p2[dec] + 1)) * n_ranks + own) * 2
           + (kind[dec] - 1))
    ukeys, first, inv = np.unique(key, return_index=True, return_inverse=True)
    n_player_h = len(ukeys)
    node_infoset[1 + dec] = inv
    h_player = (kind[dec[first]]).astype(np.int8)
    h_nact = tpl["nact"][t_idx[dec[first]]]
    # per-infoset descriptors (from the first member) for the warm-start features
    fm = dec[first]
    ti = t_idx[fm]
    inf = tpl["info"][ti]
    desc = np.full((n_player_h, 16), -1, dtype=np.int16)
    pl = kind[fm]
    desc[:, 0] = pl
    desc[:, 1] = np.where(pl == KIND_P1, r1[fm], r2[fm])
    desc[:, 2] = len(board) + inf[:, 4]
    pubs = [np.full(n_player_h, b, dtype=np.int64) for b in board] + [p1[fm], p2[fm]]
    pubs = np.stack(pubs[:3], axis=1) if len(pubs) >= 3 else np.stack(
        pubs + [np.full(n_player_h, -1)] * (3 - len(pubs)), axis=1)
    desc[:, 3:6] = pubs[:, :3]
    desc[:, 6] = inf[:, 2]
    desc[:, 7] = inf[:, 3]
    desc[:, 8] = np.where(pl == KIND_P1, inf[:, 0], inf[:, 1])
    desc[:, 9] = np.where(pl == KIND_P1, inf[:, 1], inf[:, 0])
    desc[:, 10] = stack
    desc[:, 11] = inf[:, 5]
    desc[:, 12] = tpl["depth"][ti]
    desc[:, 13] = cap
    desc[:, 14] = n_ranks
    desc[:, 15] = 0
    del key, own, inv

    # chance infosets: the root, then every chance node in id order (its own infoset)
    ch = np.flatnonzero(kind == KIND_CHANCE)
    node_infoset[0] = n_player_h
    node_infoset[1 + ch] = n_player_h + 1 + np.arange(len(ch))
    infoset_player = np.concatenate([h_player, np.zeros(1 + len(ch), dtype=np.int8)])
    ch_nact = tpl["nact"][t_idx[ch]]
    infoset_num_actions = np.concatenate([h_nact, [nd], ch_nact]).astype(np.int32)
    if deal_prob is None:
        root_p = np.full(nd, 1.0 / nd)
    else:
        root_p = np.asarray(deal_prob, dtype=np.float64)
    chance_prob = np.concatenate([root_p, 1.0 / np.repeat(ch_nact, ch_nact).astype(np.float64)])

    # payoffs
    payoff = np.zeros(n, dtype=np.float64)
    term = np.flatnonzero(kind == KIND_TERM)
    tk = tpl["term"][t_idx[term]]
    cm = tpl["commit"][t_idx[term]].astype(np.float64)
    sd = np.where(r1[term] > r2[term], 1.0, -1.0)
    payoff[1 + term] = np.where(tk == TERM_FOLD1, -cm, np.where(tk == TERM_FOLD2, cm, sd * cm))
    if scale:
        payoff /= np.abs(payoff).max()

    return Game(
        name=name or f"poker{n_ranks}r{n_rounds}c{cap}s{stack}",
        parent=parent.astype(np.int32),
        node_infoset=node_infoset.astype(np.int32),
        node_action=action.astype(np.int32),
        infoset_player=infoset_player,
        infoset_num_actions=infoset_num_actions,
        chance_prob=chance_prob,
        payoff_u1=payoff,
        payoff_u2=None,
        meta={"kind": "poker", "n_ranks": n_ranks, "n_rounds": n_rounds, "cap": cap,
              "stack": stack, "c0": c0, "board": list(board), "deals": nd, "template_nodes": tn,
              "infoset_desc": desc},
    )


def large_game() -> Game:
    """The large single-game workload: 13 ranks, 3 rounds, cap 3, stack 400 (21,509,281 nodes)."""
    return poker_game(13, 3, 3, 400, name="poker13_3r_cap3_s400")


# --------------------------------------------------------------------------- subgame family

def subgame_spec(seed: int, lo: float = 1e3, hi: float = 1e6) -> dict:
    """Draw one subgame of the batched family: a log-uniform size target in
    [lo, hi]; a start round (rounds already played) chosen at random among those
    that can reach the target, with a random prior pot and board; Dirichlet(1)
    beliefs over ranks; and the size knobs (ranks, raise cap, stack) whose node
    count lands nearest the target."""
    rng = np.random.default_rng(seed)
    target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    pots = {0: 1, 1: int(rng.choice([2, 3, 5, 7, 10])), 2: int(rng.choice([3, 5, 7, 10, 14]))}
    best_by_start = {}
    for start in (0, 1, 2):
        n_rounds, pot_c = 3 - start, pots[start]
        best = None
        for ranks in range(4, 14):
            for cap in (1, 2, 3):
                for stack in sorted({pot_c * 4, pot_c * 8, pot_c * 16, pot_c * 64, 400}):
                    nd = (ranks - start) * (ranks - start - 1)
                    size = 1 + nd * template_size(ranks, n_rounds, cap, stack, pot_c, start)
                    err = abs(math.log(size) - math.log(target))
                    if best is None or err < best[0]:
                        best = (err, start, ranks, cap, stack, size)
        best_by_start[start] = best
    good = [s for s in (0, 1, 2) if best_by_start[s][0] < math.log(1.5)]
    if good:
        start = int(rng.choice(good))
    else:
        start = min(best_by_start, key=lambda s: best_by_start[s][0])
    _, start, ranks, cap, stack, size = best_by_start[start]
    board = sorted(rng.choice(ranks, size=start, replace=False).tolist()) if start else []
    b1 = rng.dirichlet(np.ones(ranks))
    b2 = rng.dirichlet(np.ones(ranks))
    return {"seed": seed, "target": target, "start": start, "n_rounds": 3 - start,
            "c0": pots[start], "ranks": ranks, "cap": cap, "stack": stack, "size": size,
            "board": board, "b1": b1, "b2": b2}


def subgame(seed: int) -> Game:
    s = subgame_spec(seed)
    free = [r for r in range(s["ranks"]) if r not in s["board"]]
    w = np.asarray([s["b1"][a] * s["b2"][b] for a in free for b in free if a != b])
    g = poker_game(s["ranks"], s["n_rounds"], s["cap"], s["stack"], s["c0"], s["board"],
                   deal_prob=w / w.sum(), scale=True, name=f"subgame{seed}")
    g.meta.update({k: v for k, v in s.items() if k not in ("b1", "b2")})
    bel = np.zeros((2, 13), dtype=np.float32)
    bel[0, :s["ranks"]] = s["b1"]
    bel[1, :s["ranks"]] = s["b2"]
    g.meta["beliefs"] = bel
    return g

"""A second, pure-Python statement of the FACO iteration used to pin the C
oracle on tiny inputs.  Written separately from the C code: random numbers come
from numpy's own Philox generator, binary32 arithmetic from numpy float32
scalars, distances from exact integer square roots.  Far too slow for anything
but a few dozen cities."""
import math

import numpy as np

LS_2OPT, LS_OROPT, LS_SWEEP, LS_INIT_3OPT = 1, 2, 4, 8


def philox_word0(seed, ctr):
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    g = np.random.Philox(counter=(c - 1) % (1 << 256), key=int(seed))
    return int(g.random_raw(1)[0])


def dist(xy, i, j):
    dx = int(xy[i][0]) - int(xy[j][0])
    dy = int(xy[i][1]) - int(xy[j][1])
    d2 = dx * dx + dy * dy
    r = math.isqrt(d2)
    return r + (1 if d2 > r * r + r else 0)


class Ref:
    def __init__(self, xy, cl_size=16, bl_size=64, n_ants=4, min_new_edges=8,
                 rho=0.5, p_best=0.05, p_source_gbest=0.01, seed=1,
                 ls_flags=7, oropt_max_seg=3, min_new_edges_max=0):
        self.xy = [(int(a), int(b)) for a, b in xy]
        n = self.n = len(xy)
        self.k = min(cl_size, n - 1)
        self.bl = min(bl_size, n - 1 - self.k)
        self.A, self.m = n_ants, min_new_edges
        self.m_hi = min_new_edges_max
        self.rho = np.float32(rho)
        self.p_best, self.p_gb, self.seed = p_best, p_source_gbest, seed
        self.flags, self.maxseg = ls_flags, oropt_max_seg
        order = []
        for i in range(n):
            others = sorted((j for j in range(n) if j != i),
                            key=lambda j: ((self.xy[i][0] - self.xy[j][0]) ** 2 +
                                           (self.xy[i][1] - self.xy[j][1]) ** 2, j))
            order.append(others)
        self.cl = [o[:self.k] for o in order]
        self.bll = [o[self.k:self.k + self.bl] for o in order]
        self.eta = [[np.float32(1.0 / dist(self.xy, i, j)) for j in self.cl[i]] for i in range(n)]
        # initial solution: nearest neighbour from 0, then LS over all nodes
        route, vis = [0], {0}
        for _ in range(n - 1):
            u = route[-1]
            v = min((j for j in range(n) if j not in vis),
                    key=lambda j: ((self.xy[u][0] - self.xy[j][0]) ** 2 +
                                   (self.xy[u][1] - self.xy[j][1]) ** 2, j))
            route.append(v)
            vis.add(v)
        self.nn = list(route)
        init_flags = LS_2OPT | LS_SWEEP | (ls_flags & (LS_OROPT | LS_INIT_3OPT))
        route = self.local_search(route, list(range(n)), init_flags)
        self.gb = route
        self.gb_len = self.length(route)
        self.p_root = math.pow(p_best, 1.0 / n)
        self.limits()
        self.tau = [[self.tau_max] * self.k for _ in range(n)]
        self.set_source(self.gb)
        self.iter = 0
        self.delta = np.float32(0)

    # -------------------------------------------------------------------
    def length(self, r):
        return sum(dist(self.xy, r[i], r[(i + 1) % self.n]) for i in range(self.n))

    def limits(self):
        tmax = 1.0 / (float(self.gb_len) * (1.0 - float(self.rho)))
        tmin = tmax * (1.0 - self.p_root) / (float(self.k - 1) * self.p_root)
        tmin = min(tmin, tmax)
        self.tau_max, self.tau_min = np.float32(tmax), np.float32(tmin)

    def set_source(self, r):
        self.src = list(r)
        self.src_pos = {v: i for i, v in enumerate(r)}
        self.src_len = self.length(r)

    def s_succ(self, u):
        return self.src[(self.src_pos[u] + 1) % self.n]

    def s_pred(self, u):
        return self.src[(self.src_pos[u] - 1) % self.n]

    # -------------------------------------------------------------------
    def choose(self, u, vis, t, ant, step):
        row = self.cl[u]
        unv = [s for s in range(self.k) if row[s] not in vis]
        if unv:
            total = np.float32(0)
            cum = []
            for s in range(self.k):
                if row[s] not in vis:
                    total = np.float32(total + np.float32(self.tau[u][s] * self.eta[u][s]))
                cum.append(total)
            x = philox_word0(self.seed, (t, ant, step, 0))
            U = np.float32((x >> 40) / 16777216.0)
            r = np.float32(U * total)
            for s in range(self.k):
                if cum[s] > r:
                    return row[s]
            return row[unv[-1]]
        for b in self.bll[u]:
            if b not in vis:
                return b
        return min((j for j in range(self.n) if j not in vis),
                   key=lambda j: ((self.xy[u][0] - self.xy[j][0]) ** 2 +
                                  (self.xy[u][1] - self.xy[j][1]) ** 2, j))

    def threshold(self, t, ant):
        """Alg. 2's calc_num_new_edges(): the constant, or a uniform integer
        in [min_new_edges, min_new_edges_max] from the Philox word of
        (t, ant, 0, 3)."""
        if self.m_hi <= self.m:
            return self.m
        x = philox_word0(self.seed, (t, ant, 0, 3))
        return self.m + (x * (self.m_hi - self.m + 1) >> 64)

    def construct(self, t, ant):
        n = self.n
        x = philox_word0(self.seed, (t, ant, 0, 1))
        r0 = (x * n) >> 64
        route, vis, chk = [r0], {r0}, []
        new, step = 0, 0
        m = self.threshold(t, ant)
        while len(route) < n:
            u = route[-1]
            v = self.choose(u, vis, t, ant, step)
            step += 1
            route.append(v)
            vis.add(v)
            if v != self.s_succ(u) and v != self.s_pred(u):
                new += 1
                chk.append(v)
            if new >= m:
                c, app = self.s_succ(v), 0
                while c not in vis:
                    route.append(c)
                    vis.add(c)
                    c = self.s_succ(c)
                    app += 1
                if app == 0:
                    c = self.s_pred(v)
                    while c not in vis:
                        route.append(c)
                        vis.add(c)
                        c = self.s_pred(c)
        return route, chk

    # -------------------------------------------------------------------
    def best_move(self, r, pos, a, flags):
        n, xy = self.n, self.xy
        succ = lambda x: r[(pos[x] + 1) % n]
        pred = lambda x: r[(pos[x] - 1) % n]
        best = (0, None)
        if flags & LS_2OPT:
            a_s, a_p = succ(a), pred(a)
            for b in self.cl[a]:
                if dist(xy, a, a_s) > dist(xy, a, b):
                    b_s = succ(b)
                    g = dist(xy, a, a_s) + dist(xy, b, b_s) - dist(xy, a, b) - dist(xy, a_s, b_s)
                    if g > best[0]:
                        best = (g, ("2", a, a_s, b, b_s))
            for b in self.cl[a]:
                if dist(xy, a_p, a) > dist(xy, a, b):
                    b_p = pred(b)
                    g = dist(xy, a_p, a) + dist(xy, b_p, b) - dist(xy, a, b) - dist(xy, a_p, b_p)
                    if g > best[0]:
                        best = (g, ("2", a_p, a, b_p, b))
        if best[1] is None and flags & LS_OROPT:
            Lmax = min(self.maxseg, n - 3)
            for fwd in (True, False):
                for L in range(1 if fwd else 2, Lmax + 1):
                    if fwd:
                        f = l = a
                        for _ in range(L - 1):
                            l = succ(l)
                    else:
                        f = l = a
                        for _ in range(L - 1):
                            f = pred(f)
                    seg = [r[(pos[f] + i) % n] for i in range(L)]
                    p, q = pred(f), succ(l)
                    o = l if fwd else f
                    rem = dist(xy, p, a) if fwd else dist(xy, a, q)
                    base = dist(xy, p, f) + dist(xy, l, q) - dist(xy, p, q)
                    for b in self.cl[a]:
                        if b in seg or not dist(xy, a, b) < rem:
                            continue
                        for e in (succ(b), pred(b)):
                            if e in seg:
                                continue
                            g = base + dist(xy, b, e) - dist(xy, a, b) - dist(xy, o, e)
                            if g > best[0]:
                                best = (g, ("o", seg, p, q, a, b, e))
        if best[1] is None and flags & LS_INIT_3OPT:
            best = self.best_3opt(r, pos, a, best)
        return best

    def best_3opt(self, r, pos, a, best):
        """Pure 3-opt reconnection (two adjacent blocks exchange places, no
        reversal) with positive partial gains, both orientations."""
        n, xy = self.n, self.xy
        for step in (1, -1):
            nxt = lambda x: r[(pos[x] + step) % n]
            ahead = lambda frm, x: ((pos[x] - pos[frm]) * step) % n
            t1 = a
            t2 = nxt(t1)
            for t3 in self.cl[t2]:
                g1 = dist(xy, t1, t2) - dist(xy, t2, t3)
                if g1 <= 0 or t3 == t1:
                    continue
                t4 = nxt(t3)
                if t4 == t1:
                    continue
                for t5 in self.cl[t4]:
                    g2 = g1 + dist(xy, t3, t4) - dist(xy, t4, t5)
                    if g2 <= 0 or ahead(t2, t5) >= ahead(t2, t3):
                        continue
                    t6 = nxt(t5)
                    g = g2 + dist(xy, t5, t6) - dist(xy, t6, t1)
                    if g > best[0]:
                        best = (g, ("3", step, t1, t2, t3, t4, t5, t6))
        return best

    def apply(self, r, pos, mv):
        n = self.n
        if mv[0] == "2":
            _, w, x, y, z = mv
            L1 = (pos[y] - pos[x]) % n + 1
            s, L = (pos[x], L1) if 2 * L1 <= n else (pos[z], n - L1)
            idx = [(s + i) % n for i in range(L)]
            vals = [r[i] for i in idx][::-1]
            for i, v in zip(idx, vals):
                r[i] = v
                pos[v] = i
            return [w, x, y, z]
        if mv[0] == "3":
            _, step, t1, t2, t3, t4, t5, t6 = mv
            # array order: the block starting after t1 (succ) or at t3 (pred)
            first = [t2, t5] if step == 1 else [t3, t6]
            second = [t6, t3] if step == 1 else [t5, t2]
            s = pos[first[0]]
            A = [r[(s + i) % n] for i in range((pos[first[1]] - s) % n + 1)]
            B = [r[(pos[second[0]] + i) % n] for i in range((pos[second[1]] - pos[second[0]]) % n + 1)]
            for i, v in enumerate(B + A):
                r[(s + i) % n] = v
                pos[v] = (s + i) % n
            return [t1, t2, t3, t4, t5, t6]
        _, seg, p, q, a, b, e = mv
        L = len(seg)
        if r[(pos[b] + 1) % n] == e:
            x1, x2 = b, e
        else:
            x1, x2 = e, b
        # the segment joins x1 -> ... -> x2 with a next to b
        a_to_o = list(seg) if a == seg[0] else list(seg)[::-1]
        ins = a_to_o if x1 == b else a_to_o[::-1]
        D1 = (pos[x1] - pos[q]) % n + 1
        D2 = (pos[p] - pos[x2]) % n + 1
        if D1 <= D2:
            block = [r[(pos[q] + i) % n] for i in range(D1)]
            start, new = pos[seg[0]], block + ins
        else:
            block = [r[(pos[x2] + i) % n] for i in range(D2)]
            start, new = pos[x2], ins + block
        for i, v in enumerate(new):
            r[(start + i) % n] = v
            pos[v] = (start + i) % n
        return [p, q, b, e, seg[0], seg[-1]]

    def local_search(self, route, chk, flags):
        n = self.n
        r = list(route)
        pos = {v: i for i, v in enumerate(r)}
        queue, inq, touched = [], set(), set()

        def push(x):
            if x not in inq:
                inq.add(x)
                touched.add(x)
                queue.append(x)
        for c in chk:
            push(c)
        changes = 0
        while True:
            while queue and changes < n:
                a = queue.pop(0)
                inq.discard(a)
                g, mv = self.best_move(r, pos, a, flags)
                if mv is None:
                    continue
                for x in self.apply(r, pos, mv):
                    push(x)
                changes += 1
            if not (flags & LS_SWEEP) or changes >= n:
                break
            pushed = 0
            for x in sorted(touched):
                if self.best_move(r, pos, x, flags)[1] is not None:
                    push(x)
                    pushed += 1
            if pushed == 0:
                break
        return r

    # -------------------------------------------------------------------
    def run(self, iterations):
        for _ in range(iterations):
            t = self.iter + 1
            routes, lens = [], []
            for a in range(self.A):
                r, chk = self.construct(t, a)
                if self.flags & (LS_2OPT | LS_OROPT):
                    r = self.local_search(r, chk, self.flags & ~LS_INIT_3OPT)
                routes.append(r)
                lens.append(self.length(r))
            ib = min(range(self.A), key=lambda a: (lens[a], a))
            if lens[ib] < self.gb_len:
                self.gb, self.gb_len = list(routes[ib]), lens[ib]
                self.limits()
            x = philox_word0(self.seed, (t, (1 << 64) - 1, 0, 2))
            use_gb = float(x >> 40) < self.p_gb * 16777216.0
            self.set_source(self.gb if use_gb else routes[ib])
            self.delta = np.float32(1.0 / float(self.src_len))
            for i in range(self.n):
                sn, pn = self.s_succ(i), self.s_pred(i)
                for s in range(self.k):
                    j = self.cl[i][s]
                    t1 = np.float32(self.rho * self.tau[i][s])
                    t2 = np.float32(t1 + self.delta) if j in (sn, pn) else t1
                    self.tau[i][s] = max(self.tau_min, min(self.tau_max, t2))
            self.routes, self.lens = routes, lens
            self.iter = t

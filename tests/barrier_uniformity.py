"""Workgroup barriers in divergent control flow, from LLVM's uniformity
printout (opt -passes='print<uniformity>').

The ant kernels with several waves per ant synchronise their waves with
s_barrier.  A barrier reached under a branch the compiler lowers with an exec
mask (a divergent branch) could run with no active lane while the other waves
wait elsewhere, and the team's commands would pair up wrongly.  This module
parses the printout, builds the control-flow graph of the kernel, computes
post-dominators, and lists every block with a barrier that lies between a
divergent branch and that branch's immediate post-dominator."""
import re
import sys


def check(text):
    """Returns (stats dict, list of (barrier block, divergent branch blocks))."""
    txt = text.split("\n")
    blocks, order = {}, []
    cur = None
    mode = None
    nfunc = 0
    for line in txt:
        if line.startswith("UniformityInfo for function"):
            nfunc += 1
            if nfunc > 1:  # one function per printout
                break
        m = re.match(r"^BLOCK (\S+)", line)
        if m:
            cur = m.group(1); order.append(cur)
            blocks[cur] = {"succ": [], "div": False, "bar": False, "term": ""}
            mode = None
            continue
        if cur is None:
            continue
        if line.startswith("END BLOCK"):
            cur = None; continue
        if line.startswith("DEFINITIONS"):
            mode = "def"; continue
        if line.startswith("TERMINATORS"):
            mode = "term"; continue
        if "llvm.amdgcn.s.barrier" in line:
            blocks[cur]["bar"] = True
        if mode == "term":
            blocks[cur]["term"] += line
            blocks[cur]["succ"] += re.findall(r"label %(\S+?)[\s,\]]", line + " ")
            if line.strip().startswith("DIVERGENT:") and ("br i1" in line or "switch" in line):
                blocks[cur]["div"] = True
    for b in blocks.values():
        b["succ"] = list(dict.fromkeys(s for s in b["succ"] if s in blocks))
    entry = order[0]
    # post-dominators (iterative, on reverse postorder of the reverse graph)
    EXIT = "__exit__"
    preds = {b: [] for b in blocks}
    for b, d in blocks.items():
        for s in d["succ"]:
            preds[s].append(b)
    exits = [b for b, d in blocks.items() if not d["succ"]]
    rsucc = {EXIT: exits}
    for b in blocks:
        rsucc[b] = preds[b]
    # reverse postorder from EXIT in reverse graph
    seen, post = set(), []
    stack = [(EXIT, iter(rsucc[EXIT]))]
    seen.add(EXIT)
    while stack:
        node, it = stack[-1]
        nxt = next(it, None)
        if nxt is None:
            post.append(node); stack.pop()
        elif nxt not in seen:
            seen.add(nxt); stack.append((nxt, iter(rsucc[nxt])))
    rpo = post[::-1]
    idx = {b: i for i, b in enumerate(rpo)}
    ipdom = {EXIT: EXIT}
    def intersect(a, b):
        while a != b:
            while idx[a] > idx[b]:
                a = ipdom[a]
            while idx[b] > idx[a]:
                b = ipdom[b]
        return a
    changed = True
    while changed:
        changed = False
        for b in rpo[1:]:
            # predecessors in reverse graph = successors in CFG (plus EXIT for exits)
            ps = list(blocks[b]["succ"]) if b in blocks else []
            if b in exits:
                ps = ps + [EXIT]
            ps = [p for p in ps if p in ipdom]
            if not ps:
                continue
            new = ps[0]
            for p in ps[1:]:
                new = intersect(p, new)
            if ipdom.get(b) != new:
                ipdom[b] = new; changed = True
    unreached = [b for b in blocks if b not in ipdom]
    divregion = {}
    for b, d in blocks.items():
        if not d["div"]:
            continue
        stop = ipdom.get(b)
        st = list(d["succ"])
        vis = set()
        while st:
            x = st.pop()
            if x == stop or x in vis:
                continue
            vis.add(x)
            st.extend(blocks[x]["succ"])
        for x in vis:
            divregion.setdefault(x, []).append(b)
    bars = [b for b, d in blocks.items() if d["bar"]]
    bad = [b for b in bars if b in divregion]
    stats = {"blocks": len(blocks), "divergent_branches": sum(d["div"] for d in blocks.values()),
             "barriers": len(bars), "unreached": len(unreached)}
    return stats, [(b, divregion[b]) for b in bad]


if __name__ == "__main__":
    st, bad = check(open(sys.argv[1]).read())
    print(st, "barriers under divergent branches:", len(bad))
    for b, brs in bad:
        print("  block", b, "under", brs[:6])

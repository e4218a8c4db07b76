"""Seeded formula texts for the evaluation workloads.

Text generation only: nothing here evaluates the formulas.  The language is
the ImgQL subset accepted by both the library and the oracle:

    let NAME = expr            output "name" expr
    expr: a | b, a & b, !a, (e), true, false,
          intensity(img[, c]) >. t   (also <., >=., <=.),
          threshold t: a number or percentile(img, c, q),
          near(e), N(e), interior(e), reach(a, b), surrounded(a, b), grow(a, b),
          user macros  let f(x, y) = expr.
"""
import numpy as np

PLAIN_FORMULA = """\
// 12-node formula over one smoothed-noise channel
let A  = intensity(img) >. 0.65
let B  = intensity(img) >. 0.35
let C  = intensity(img) <. 0.45
let nA = !A
let D  = B & nA
let E  = D | C
let F  = near(A)
let G  = near(E)
let R1 = reach(A, B)
let R2 = reach(C, nA)
let S  = surrounded(F, B)
let O  = R1 | S
output "G" G
output "R2" R2
output "O" O
"""

# The shape of the paper's brain-tumour specification (Fig. specification):
# two intensity thresholds and grow.  Thresholds are fractions of the range.
GROW_SPEC = """\
let hI = intensity(img) >. {hi}
let vI = intensity(img) >. {lo}
let gtv = grow(hI, vI)
output "segmentation" gtv
"""

# Arithmetic atoms (the tool's built-in arithmetic) and touch on two
# channels, thresholds as fractions of a [0, 1) range.
ARITH_FORMULA = """\
let A = (intensity(img, 0) + intensity(img, 1)) * 0.5 >. {t0}
let B = intensity(img, 0) - intensity(img, 1) <. {t1}
let C = abs(intensity(img, 1) - 0.5) * 2 <=. {t2}
let D = intensity(img, 0) / (intensity(img, 1) + 0.25) >=. 1
let E = min(intensity(img, 0), intensity(img, 1)) >. max(0.2, percentile(img, 1, 0.4) - 0.1)
let F = intensity(img, 0) >. percentile(img, 0, 0.6)
output "a" A
output "b" B & !C
output "d" D | E
output "touch" touch(A, C)
output "touch2" touch(!B, F & D)
output "mix" grow(E, A | B) & near(touch(C, D))
output "neg" -intensity(img, 1) <. -{t3}
"""

# A segmentation-shaped formula for volumes (two channels in [0, ~1.2]):
# thresholds, percentiles, arithmetic, N, interior and every reach-type
# operator.
VOLUME_FORMULA = """\
let A = intensity(img, 0) >. percentile(img, 0, 0.95)
let B = intensity(img, 0) >. percentile(img, 0, 0.86)
let C = intensity(img, 1) >. 0.5
let M = (intensity(img, 0) + intensity(img, 1)) * 0.5 >. 0.45
let core = grow(A, B)
output "core" core
output "edema" grow(core, B | (C & M)) & !core
output "shell" near(core) & !interior(core)
output "enclosed" surrounded(C, near(core))
output "contact" touch(C, core)
output "reach" reach(A, M)
"""

REACH_OPS = ("reach", "surrounded", "grow")


class _Dag:
    def __init__(self, rng):
        self.rng = rng
        self.lines = []
        self.names = []
        self.unused = []      # names not yet consumed, oldest first
        self.marked = []      # nodes always emitted as outputs
        self.n_nodes = 0

    def add(self, expr, cost=1):
        name = f"n{len(self.names)}"
        self.lines.append(f"let {name} = {expr}")
        self.names.append(name)
        self.unused.append(name)
        self.n_nodes += cost
        return name

    def pick(self, exclude=()):
        """An operand: an unconsumed node if any (oldest-first with some
        randomness), else a recent node."""
        rng = self.rng
        cand = [u for u in self.unused if u not in exclude]
        if cand and rng.random() < 0.7:
            k = min(len(cand), 4)
            name = cand[int(rng.integers(0, k))]
        else:
            pool = [n for n in self.names[-24:] if n not in exclude] or self.names
            name = pool[int(rng.integers(0, len(pool)))]
        if name in self.unused:
            self.unused.remove(name)
        return name

    def text(self, max_outputs=16):
        outs = list(self.marked)
        for u in reversed(self.unused):
            if len(outs) >= max_outputs:
                break
            if u not in outs:
                outs.append(u)
        if self.names[-1] not in outs:
            outs.append(self.names[-1])
        body = "\n".join(self.lines)
        tail = "\n".join(f'output "{o}" {o}' for o in outs)
        return body + "\n" + tail + "\n"


def _grow_ops(d, n_nodes, reach_slots, extra_atom):
    """Add binary/unary operator nodes until `n_nodes`, putting reach-type
    nodes at the positions in `reach_slots` (by node count)."""
    rng = d.rng
    slots = sorted(reach_slots)
    kinds = ["and", "or", "not", "near", "interior", "andnot"]
    weights = np.array([0.24, 0.2, 0.12, 0.2, 0.08, 0.16])
    while d.n_nodes < n_nodes:
        if slots and d.n_nodes >= slots[0]:
            slots.pop(0)
            op = REACH_OPS[int(rng.integers(0, 3))]
            a = d.pick()
            b = d.pick(exclude=(a,))
            d.marked.append(d.add(f"{op}({a}, {b})"))
            continue
        if extra_atom is not None and rng.random() < 0.08:
            d.add(extra_atom(rng))
            continue
        k = kinds[int(rng.choice(len(kinds), p=weights))]
        if k in ("and", "or"):
            a = d.pick()
            b = d.pick(exclude=(a,))
            d.add(f"{a} {'&' if k == 'and' else '|'} {b}")
        elif k == "andnot":
            a = d.pick()
            b = d.pick(exclude=(a,))
            d.add(f"{a} & !{b}", cost=2)
        elif k == "not":
            d.add(f"!{d.pick()}")
        elif k == "near":
            d.add(f"near({d.pick()})")
        else:
            d.add(f"interior({d.pick()})")


def ellipse_dag(seed=2, n_nodes=100, n_reach=10, n_ellipses=200):
    """Formula over the three-channel ellipse/maze image: intensity-window
    atoms select single ellipses on channel 0, the first reach-type node is
    reach(seed, maze), and `n_reach` reach/surrounded/grow nodes in total."""
    rng = np.random.default_rng(seed)
    d = _Dag(rng)
    maze = d.add("intensity(img, 1) >. 0.5")
    seed_px = d.add("intensity(img, 2) >. 0.5")
    d.unused.remove(maze)
    d.unused.remove(seed_px)
    first = d.add(f"reach({seed_px}, {maze})")
    corridor = d.add(f"grow({seed_px}, {maze})")
    d.marked += [first, corridor]
    step = 1.0 / (2.0 * n_ellipses)
    chosen = rng.choice(n_ellipses, size=8, replace=False)
    for j in chosen:
        v = 0.5 + (j + 1) * step
        lo = d.add(f"intensity(img) >. {v - step / 2:.6f}")
        hi = d.add(f"intensity(img) <. {v + step / 2:.6f}")
        d.unused.remove(lo)
        d.unused.remove(hi)
        d.add(f"{lo} & {hi}")
    for t in (0.12, 0.25, 0.4):
        d.add(f"intensity(img) <. {t}")
    d.add("intensity(img) >. 0.5")

    def extra(r):
        return f"intensity(img) {'>.' if r.random() < 0.5 else '<.'} {r.uniform(0.05, 0.95):.5f}"

    slots = np.linspace(d.n_nodes + 4, n_nodes - 4, n_reach - 2).astype(int).tolist()
    _grow_ops(d, n_nodes, slots, extra)
    return d.text()


def chain_dag(seed=3, n_chain=10000, n_reach=500, kmax=50):
    """Long sequential formula over a random 0/1 mask.  x_0 = (m >. 0); then
    the chain rotates through N x_{i-1}, x_{i-1} & x_j, !x_{i-1}, where the
    partner x_j is drawn from the previous kmax elements (j <= i-2) among
    x_0 and the & and ! elements, so hash-consing cannot merge elements and
    the density does not collapse to all-0 or all-1.  After every
    n_chain/n_reach rotation steps one more element reach(x_{i-1}, x_j) is
    inserted and the rotation resumes at &.  Outputs: every 1000th element
    and the last one."""
    rng = np.random.default_rng(seed)
    lines = ["let x0 = intensity(img) >. 0"]
    partners = [0]            # indices of x0, & and ! elements
    every = max(1, n_chain // max(1, n_reach))
    i, rot, made_chain, made_reach, since = 0, 0, 0, 0, 0
    outs = []

    def partner(i):
        lo = i - kmax
        cand = [j for j in partners[-64:] if lo <= j <= i - 2]
        if not cand:
            cand = [partners[-1]] if partners[-1] <= i - 2 else [0]
        return cand[int(rng.integers(0, len(cand)))]

    while made_chain < n_chain or made_reach < n_reach:
        i += 1
        if made_reach < n_reach and since >= every and i >= 3:
            lines.append(f"let x{i} = reach(x{i - 1}, x{partner(i)})")
            made_reach += 1
            since = 0
            rot = 1
        else:
            r = rot % 3
            rot += 1
            if r == 0:
                lines.append(f"let x{i} = near(x{i - 1})")
            elif r == 1:
                lines.append(f"let x{i} = x{i - 1} & x{partner(i)}")
                partners.append(i)
            else:
                lines.append(f"let x{i} = !x{i - 1}")
                partners.append(i)
            made_chain += 1
            since += 1
        if i % 1000 == 0:
            outs.append(i)
    outs.append(i)
    tail = "\n".join(f'output "x{o}" x{o}' for o in sorted(set(outs)))
    return "\n".join(lines) + "\n" + tail + "\n"


def segmentation_dag(seed=4, n_nodes=60, channels=4):
    """Shared segmentation-style formula for the uneven batch: per-channel
    percentile thresholds (q in {0.95, 0.86, 0.5, 0.3}, the first two as in
    the paper's specification), then near, reach, grow and surrounded."""
    rng = np.random.default_rng(seed)
    d = _Dag(rng)
    for c in range(channels):
        hi = d.add(f"intensity(img, {c}) >. percentile(img, {c}, 0.95)")
        lo = d.add(f"intensity(img, {c}) >. percentile(img, {c}, 0.86)")
        d.unused.remove(hi)
        d.unused.remove(lo)
        d.add(f"grow({hi}, {lo})")
    for c in range(channels):
        d.add(f"intensity(img, {c}) <. percentile(img, {c}, 0.3)")

    def extra(r):
        c = int(r.integers(0, channels))
        q = float(r.choice([0.5, 0.7, 0.9]))
        return f"intensity(img, {c}) >. percentile(img, {c}, {q})"

    slots = np.linspace(d.n_nodes + 3, n_nodes - 2, 6).astype(int).tolist()
    _grow_ops(d, n_nodes, slots, extra)
    return d.text(max_outputs=8)


def random_dag(seed, n_nodes, n_reach, channels=1, max_outputs=8):
    """Random formula over `channels` float channels in [0, 1], used for
    request streams and fuzzing."""
    rng = np.random.default_rng(seed)
    d = _Dag(rng)

    def extra(r):
        c = int(r.integers(0, channels))
        op = [">.", "<.", ">=.", "<=."][int(r.integers(0, 4))]
        return f"intensity(img, {c}) {op} {r.uniform(0.05, 0.95):.5f}"

    for _ in range(min(3, n_nodes)):
        d.add(extra(rng))
    slots = (np.linspace(d.n_nodes + 1, max(d.n_nodes + 1, n_nodes - 1), n_reach).astype(int)
             .tolist() if n_reach > 0 else [])
    _grow_ops(d, n_nodes, slots, extra)
    return d.text(max_outputs=max_outputs)


SERVE_SIDES = (256, 512, 1024, 2048, 4096, 8192)


def serve_formulas(seed=5, n_random=5, n_max=2000, reach_max=50):
    """Formula texts of the serving mix: `n_random` formulas with node counts
    log-uniform in [20, n_max] and U{0 .. min(reach_max, n/10)} reach-type
    nodes, plus one formula at the top of both ranges (n_max nodes, reach_max
    reach-type nodes).  Returns [(text, n_nodes, n_reach)]."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_random):
        n = int(round(np.exp(rng.uniform(np.log(20), np.log(n_max)))))
        specs.append((n, int(rng.integers(0, min(reach_max, n // 10) + 1))))
    specs.append((n_max, reach_max))
    return [(random_dag(500 + k, n_nodes=n, n_reach=r), n, r) for k, (n, r) in enumerate(specs)]

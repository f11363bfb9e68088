"""bench.py's command line on the CPU: the parser builds (every workload
name is offered) and a request for more than one GPU is refused with a
message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, timeout=300)


def test_help_lists_workloads():
    r = _bench("--help")
    assert r.returncode == 0, r.stderr
    for name in ("plain", "generation", "uneven", "precision", "serving", "reward"):
        assert name in r.stdout


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "single" in r.stderr, r.stderr


def _executed_by_tree(prog):
    """Nodes one case evaluates after constant subtrees fold, by recursion
    over the expression tree: (count, is_constant) of a subtree."""
    stack = []
    for t in prog:
        op = int(t) & 0xFF
        if op <= 1:
            stack.append((1 if op == 0 else 0, op == 1))
        elif op >= 6:
            n, c = stack.pop()
            stack.append((n if c else n + 1, c))
        else:
            nb, cb = stack.pop()
            na, ca = stack.pop()
            if ca and cb:
                stack.append((0, True))
            else:
                stack.append(((1 if ca else na) + (1 if cb else nb) + 1, False))
    n, c = stack[0]
    return 1 if c else n


def test_executed_node_counts_match_a_tree_walk():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=3000, n_cases=16)
    got = bench.executed_node_counts(w.pop.nodes, w.pop.offsets, chunk=700)
    want = np.array([_executed_by_tree(w.pop.nodes[w.pop.offsets[p]:w.pop.offsets[p + 1]])
                     for p in range(w.pop.n_programs)])
    assert np.array_equal(got, want)
    # hand-made cases: x0 c + (3), c c + (1), c sin x0 * (3), x0 c c + * (3), c (1)
    C = lambda j: 1 | (j << 8)
    progs = [[0, C(0), 2], [C(0), C(1), 2], [C(0), 6, 0, 4], [0, C(0), C(1), 2, 4], [C(0)]]
    nodes = np.array([t for q in progs for t in q], np.uint32)
    off = np.cumsum([0] + [len(q) for q in progs])
    assert list(bench.executed_node_counts(nodes, off)) == [3, 1, 3, 3, 1]


def _operators_by_tree(prog, by_op):
    """Operators that depend on a variable, by recursion over the expression
    tree (a subtree is a constant flag)."""
    stack = []
    for t in prog:
        op = int(t) & 0xFF
        if op <= 1:
            stack.append(op == 1)
        elif op >= 6:
            c = stack.pop()
            if not c:
                by_op[op] += 1
            stack.append(c)
        else:
            cb, ca = stack.pop(), stack.pop()
            if not (ca and cb):
                by_op[op] += 1
            stack.append(ca and cb)


def test_executed_operator_mix_matches_a_tree_walk():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    from paper_2607_06731_amd import synth
    w = synth.make_workload("generation", n_programs=3000, n_cases=16)
    sel = np.arange(w.pop.n_programs) % 3 != 1
    got = bench.executed_operator_mix(w.pop.nodes, w.pop.offsets, sel, chunk=700)
    want = np.zeros(12, np.int64)
    for p in np.nonzero(sel)[0]:
        _operators_by_tree(w.pop.nodes[w.pop.offsets[p]:w.pop.offsets[p + 1]], want)
    assert np.array_equal(got, want)
    # hand-made: x0 c + (one +), c c + (none), c sin x0 * (one *), x0 sin c sin * (sin, *)
    C = lambda j: 1 | (j << 8)
    progs = [[0, C(0), 2], [C(0), C(1), 2], [C(0), 6, 0, 4], [0, 6, C(0), 6, 4]]
    nodes = np.array([t for q in progs for t in q], np.uint32)
    off = np.cumsum([0] + [len(q) for q in progs])
    mix = bench.executed_operator_mix(nodes, off, np.ones(4, bool))
    assert list(mix) == [0, 0, 1, 0, 2, 0, 1, 0, 0, 0, 0, 0]


def test_code_digest_ignores_comments_and_layout_only():
    sys.path.insert(0, ROOT)
    import bench
    a = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    b = "/* the successor */\nint f(int x) { return x + 1; }\n"
    c = "int f(int x)\n{\n    return x + 2;\n}\n"
    assert bench.code_digest([a]) == bench.code_digest([b])
    assert bench.code_digest([a]) != bench.code_digest([c])
    assert bench.code_digest([a, c]) != bench.code_digest([c, a])

"""Recipe that wrote ``dolphins_edges.txt`` and ``karate_edges.txt``.

Both graphs are drawn in the paper's Figure 1 (the introduction's worked
example) as TikZ pictures whose ``\\foreach \\startnode/\\endnode in {...}``
lists are the edge lists.  The figure prints their von Neumann graph entropy
(dolphins 3.846, karate 3.154).  This script reads the paper's LaTeX source and
writes one ``u v`` pair per line; it is run once by hand, never by the tests.

Usage:  python tests/golden/extract_fig1.py <path to the paper's LaTeX source>
"""
import re
import sys
from pathlib import Path


def edge_blocks(tex):
    # every edge list in the source, in order of appearance
    pat = re.compile(r"\\foreach \\startnode/\\endnode in \{(.*?)\}", re.S)
    return [m.group(1) for m in pat.finditer(tex)]


def parse(block):
    pairs = []
    for item in block.split(","):
        item = item.strip()
        if not item:
            continue
        a, b = item.split("/")
        pairs.append((int(a.strip().lstrip("n")), int(b.strip().lstrip("n"))))
    return pairs


def main(src):
    tex = Path(src).read_text()
    blocks = edge_blocks(tex)
    assert len(blocks) == 2, len(blocks)
    out = Path(__file__).parent
    # first picture: dolphins, nodes named n1..n62 -> ids 0..61
    dol = [(a - 1, b - 1) for a, b in parse(blocks[0])]
    # second picture: karate, nodes named 0..33
    kar = parse(blocks[1])
    for name, edges, nodes, cite in (
        ("dolphins", dol, 62, "Figure 1, first TikZ picture (nodes renumbered n1..n62 -> 0..61)"),
        ("karate", kar, 34, "Figure 1, second TikZ picture (nodes 0..33)"),
    ):
        hdr = [
            f"# {name}: undirected edge list, {nodes} nodes, {len(edges)} edges",
            f"# source: arXiv 2003.01282 (SLaQ, WWW'20), {cite}",
            f"# the figure prints VNGE {'3.846' if name == 'dolphins' else '3.154'}"
            " (combinatorial Laplacian, natural log)",
        ]
        lines = hdr + [f"{a} {b}" for a, b in edges]
        (out / f"{name}_edges.txt").write_text("\n".join(lines) + "\n")
        print(name, nodes, len(edges))


if __name__ == "__main__":
    main(sys.argv[1])

"""The selection rules against a worked example written out by hand
(tests/golden/krum_worked_example.txt; Appendix, "Descriptions of Aggregation
Rules", and Algorithm 2).  Both the oracle's rules and the product's
(paper_2408_06197_amd/robust.py) must reproduce every score and choice; a
neighbour count of n - c - 1 or n - c - 3, or a 0-based Median index, fails."""
import pathlib

import numpy as np

from paper_2408_06197_amd import robust

GOLDEN = pathlib.Path(__file__).parent / "golden" / "krum_worked_example.txt"


def load():
    rows, cases = [], []
    for line in GOLDEN.read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "matrix":
            rows.append([float(x) for x in tok[1:]])
        elif tok[0] == "case":
            n, c, l = int(tok[1]), int(tok[2]), int(tok[3])
            i = tok.index("scores")
            k = tok.index("krum")
            m = tok.index("median")
            mk = tok.index("multikrum")
            cases.append(dict(n=n, c=c, l=l, scores=[float(x) for x in tok[i + 1:k]], krum=[int(tok[k + 1])],
                              median=[int(tok[m + 1])], multikrum=[int(x) for x in tok[mk + 1:]]))
    return np.array(rows), cases


def test_oracle_rules_match_worked_example(oracle_mod):
    O = oracle_mod
    D6, cases = load()
    for cs in cases:
        D = D6[: cs["n"], : cs["n"]]
        assert np.array_equal(O.krum_scores(D, cs["c"]), cs["scores"])
        assert O.select("krum", D, cs["c"]) == cs["krum"]
        assert O.select("median", D, cs["c"]) == cs["median"]
        assert O.select("multikrum", D, cs["c"], cs["l"]) == cs["multikrum"]


def test_product_rules_match_worked_example():
    D6, cases = load()
    for cs in cases:
        D = D6[: cs["n"], : cs["n"]]
        iu = np.triu_indices(cs["n"], k=1)
        assert np.array_equal(robust.distance_matrix(D[iu], cs["n"]), D)
        assert np.array_equal(robust.krum_scores(D, cs["c"]), cs["scores"])
        for rule in robust.RULES:
            assert robust.select(rule, D, cs["c"], cs["l"]) == cs[rule], rule

"""N_st pins: the stratification counts the paper states (tests/golden/nst_cases.json)."""
import json
import os

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nst_cases.json")


def test_vegasp_nst_cases(orc):
    cases = json.load(open(GOLD))
    for c in cases["vegasp"]:
        assert orc.nst(c["dim"], c["n_ev"]) == c["n_st"], c


def test_classic_nst_case(orc):
    for c in json.load(open(GOLD))["classic"]:
        n = orc.nst_classic(c["dim"], c["n_ev"])
        assert n == c["n_st"]
        assert c["n_ev"] // n ** c["dim"] == c["per_hypercube"]


def test_nst_is_the_largest_admissible(orc):
    # brute force over small cases: largest n >= 1 with 4 n^D <= N_ev
    for dim in range(1, 7):
        for n_ev in list(range(1, 300)) + [4 * 7 ** dim, 4 * 7 ** dim - 1]:
            want = 1
            while 4 * (want + 1) ** dim <= n_ev:
                want += 1
            assert orc.nst(dim, n_ev) == want, (dim, n_ev)

"""Values the paper prints, held in tests/golden/paper_constants.json."""
import json
import os

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_oracle_line_search_candidates_are_the_papers(orc):
    # Sec. IV "Forward pass with line-search": alpha in {1.0, 0.5, 0.25, 0.1},
    # read from the C oracle that uses them, in the order it tries them
    assert list(orc.alphas()) == GOLD["line_search_alphas"]


def test_table1_derived_throughput():
    # solves/s = B / (fwd + bwd) derived from Table I, used as context in the bench report
    rows = {(r["B"], r["T"]): r for r in GOLD["table1_ms"]}
    r = rows[(256, 10)]
    assert round(256 / ((r["ca_fwd"] + r["ca_bwd"]) * 1e-3)) == 100392

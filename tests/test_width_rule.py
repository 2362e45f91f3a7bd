"""The block-width rule of the Jacobi rounds (no GPU): the table the tuner
measured on MI355X is the rule its own derivation gives, monotone, and the
library's default."""
import json
import os
import re

from paper_1910_09142_amd import tune_width

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_table_is_the_measured_rule():
    with open(tune_width.OUT) as f:
        table = json.load(f)
    measured = {int(c): {int(b): v for b, v in m.items()}
                for c, m in table["measured"].items()}
    assert tune_width.derive_rule(measured) == table["rule"]
    rule = table["rule"]
    assert all(a[0] < b[0] and a[1] >= b[1] for a, b in zip(rule, rule[1:]))
    assert all(n >= 512 and c >= 1 for n, c in rule)
    # the library's default rule (hmps.cpp) is this table
    with open(os.path.join(ROOT, "paper_1910_09142_amd", "csrc",
                           "hmps.cpp")) as f:
        src = f.read()
    body = re.search(r"DEFAULT_WIDTH_RULE\[\] = \{(.*?)\};", src, re.S).group(1)
    entries = [[int(a), int(b)]
               for a, b in re.findall(r"\{(\d+),\s*(\d+)\}", body)]
    assert entries == rule


def test_rule_derivation():
    # wide wins from 16 chains on at 768 vectors, never at 540; a larger
    # size never needs more chains than a smaller one
    m = {180: {8: [10, 9], 64: [10, 9]},
         256: {8: [10, 9], 16: [10, 11], 64: [10, 12]},
         384: {8: [10, 9], 16: [10, 9], 32: [10, 11], 64: [10, 12]}}
    assert tune_width.derive_rule(m) == [[768, 16], [1152, 16]]

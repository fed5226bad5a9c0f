"""What the paper fixes, written out from its statements (no oracle code here).

* Theorem 1 (Section 3.2): the complete list of pairs of both kinds with n < 1.4e12:
  first kind (75, 1215) and m = 2^k - 2, n = 2^(2k) - 2^(k+1) for 2 <= k <= 20;
  second kind (35, 4374) and m = 2^k + 1, n = 2^(2k) + 2^(k+1) for 0 <= k <= 20.
* Tables 1 and 2 (Section 3.2) with their printed factorizations (tests/golden/).
"""
import os

THEOREM1_LIMIT = 14 * 10**11  # 1.4e12


def theorem1_pairs(limit_n):
    """Sorted (m, n, kind) of Theorem 1 with n <= limit_n (limit_n < 1.4e12)."""
    assert limit_n < THEOREM1_LIMIT
    out = []
    if 1215 <= limit_n:
        out.append((75, 1215, 1))
    if 4374 <= limit_n:
        out.append((35, 4374, 2))
    for k in range(2, 21):
        m, n = 2**k - 2, 2**(2 * k) - 2**(k + 1)
        if n <= limit_n:
            out.append((m, n, 1))
    for k in range(0, 21):
        m, n = 2**k + 1, 2**(2 * k) + 2**(k + 1)
        if n <= limit_n:
            out.append((m, n, 2))
    return sorted(out)


def parse_factorization(s):
    """'2^3*3*5^2' -> {2: 3, 3: 1, 5: 2}."""
    out = {}
    for tok in s.strip().split("*"):
        if "^" in tok:
            p, e = tok.split("^")
            out[int(p)] = out.get(int(p), 0) + int(e)
        else:
            out[int(tok)] = out.get(int(tok), 0) + 1
    return out


def load_table(path):
    """Rows of (m, n, [fact strings in printed column order])."""
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, *facts = [c.strip() for c in line.split("|")]
            m, n = (int(v) for v in head.split())
            rows.append((m, n, [parse_factorization(fs) for fs in facts]))
    return rows


def golden(name):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)

"""Plant plausible mistakes in the oracle (on the CPU) and check the pins see them.

Each mutant is oracle/oracle.c with one textual change, compiled into a
temporary library.  The checks below are the same independent references the
other oracle tests use (enumeration, the Kronecker-built Hamiltonian, the
paper's worked examples); every mutant must fail at least one of them.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import brute, core

SRC = os.path.join(os.path.dirname(core.__file__), "oracle.c")

MUTANTS = {
    "diagonal_sign": ("diag += -Juv * mu * mv;", "diag += Juv * mu * mv;"),
    "dropped_half": ("y += -0.5 * Juv * f * x_at(x, j);\n            }\n            /* s-(u) s+(v) */",
                     "y += -1.0 * Juv * f * x_at(x, j);\n            }\n            /* s-(u) s+(v) */"),
    "ladder_factor": ("sqrt((double)cur[u] * (two_s - cur[u] + 1)) *",
                      "sqrt((double)cur[u] * (two_s - cur[u])) *"),
    "rank_off_by_one": ("index += below(D, N, two_s, k, T, digit);",
                        "index += below(D, N, two_s, k, T, digit + 1);"),
    "rank_wrong_prefix": ("index += below(D, N, two_s, k, T, digit);",
                          "index += below(D, N, two_s, k, T - digit, digit);"),
    "block_wrong_row": ("start += count_at(D, N, two_s, k - 1, T - m);",
                        "start += count_at(D, N, two_s, k, T - m);"),
    "unrank_boundary": ("if (below(D, N, two_s, k, T, n) <= r)",
                        "if (below(D, N, two_s, k, T, n) < r)"),
    "count_recursion": ("for (int k = 0; k <= two_s; ++k) {\n                int prev",
                        "for (int k = 0; k < two_s; ++k) {\n                int prev"),
    "successor_refill": ("int put = balls < two_s ? balls : two_s;",
                         "int put = balls < two_s - 1 ? balls : (two_s > 1 ? two_s - 1 : 1);"),
    "second_ladder_dropped": ("                y += -0.5 * Juv * f * x_at(x, j);\n            }\n        }\n    }",
                              "                y += 0.0 * Juv * f * x_at(x, j);\n            }\n        }\n    }"),
    "swapped_sites": ("work[u] -= 1;\n                work[v] += 1;",
                      "work[u] += 1;\n                work[v] -= 1;"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = os.path.join(tmpdir, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmpdir, f"{name}.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", lib, path,
                    "-lm"], check=True)
    return core.bind(lib)


def _pins_pass(lib):
    """True if every independent check passes with this oracle library."""
    try:
        # count table vs enumeration
        for N, two_s in ((4, 2), (3, 3), (5, 1)):
            D = core.count_table(N, two_s, lib)
            for A in range(N * two_s + 1):
                if D[N, A] != brute.count_by_enumeration(N, two_s, A):
                    return False
        # codec and successor vs enumeration
        for N, two_s in ((6, 1), (4, 2), (3, 3)):
            for A in range(N * two_s + 1):
                digits, _ = brute.enumerate_subspace(N, two_s, A)
                sub = core.Subspace(N, two_s, A, lib=lib)
                if sub.dim != digits.shape[0]:
                    return False
                for i in range(sub.dim):
                    if not np.array_equal(sub.unrank(i), digits[i]):
                        return False
                    if sub.rank(digits[i]) != i:
                        return False
                    if i + 1 < sub.dim:
                        nxt = sub.successor(digits[i])
                        if nxt is None or not np.array_equal(nxt, digits[i + 1]):
                            return False
        # H x vs the Kronecker-built block
        rng = np.random.default_rng(0)
        for N, two_s in ((5, 1), (4, 2), (3, 3)):
            J = rng.normal(size=(N, N))
            J = np.triu(J, 1)
            J = J + J.T
            for A in range(N * two_s + 1):
                sub = core.Subspace(N, two_s, A, lib=lib)
                block = brute.subspace_hamiltonian(N, two_s, A, J)
                x = rng.uniform(-1, 1, sub.dim)
                if np.abs(sub.apply(J, x) - block @ x).max() > 1e-12:
                    return False
    except (IndexError, ValueError, RuntimeError, OverflowError):
        return False
    return True


def test_unmutated_oracle_passes():
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "clean.so")
        subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", path,
                        SRC, "-lm"], check=True)
        assert _pins_pass(core.bind(path))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        assert not _pins_pass(_build_mutant(name, d)), f"mutant {name} survived"

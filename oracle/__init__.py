"""CPU oracle for the degenerate-primer scan, melting temperature and pairing.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (``paper_2509_13300_amd``) never imports it, and
this package imports nothing from the product path: the two share no code,
tables or constants.  Both are fed by the seeded generator in ``synth``.

What it computes, and where the paper defines it (AmpliconHunter,
arXiv 2509.13300):

* ``iupac``  -- degenerate primers as mixtures of oligonucleotides over the
  IUPAC alphabet (Section 1, Introduction).
* ``scan``   -- binding sites with at most k mismatches on both strands and a
  3'-clamp post-filter (Section 2.1, "Primer matching"); plus a brute-force
  checker that enumerates every oligo of the expansion.
* ``tm``     -- nearest-neighbour melting temperature of every compatible
  oligo, maximum per site (Section 2.1, "Melting temperature filtering").
* ``pair``   -- opposite-strand pairing within a length window and FR / RF /
  FF / RR labels (Section 2.1, "Amplicon calling" and "Amplicon analysis").

Arithmetic is float64.  Readings of the paper where it is silent are listed
in the module docstrings (R-numbers) and in the design notes.

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
brute force, closed forms, invariants and values derived by hand, except the
melting temperature of *mismatched* duplexes, whose published tables are not
available here: "parity unpinned" against the paper's tool for that case (its
model here is the declared mismatch-zero reading, pinned only by invariants).
"""

"""Runs the oracle's pins against one build of the C oracle.

Usage: python oracle_battery.py LIBRARY.  Exit status 0 when every pin of
test_oracle_pins passes with the oracle module pointed at LIBRARY, 1 when one
fails (the failing pin is printed).  The planted-mistake tests run this in a
subprocess for each broken copy of the oracle, so that a copy that crashes
cannot take the test session down.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def battery():
    """(name, callable taking the oracle module) for every pin."""
    import test_oracle_pins as pins
    out = []
    for n in (1, 2, 3, 5, 8, 10):
        out.append(("exhaustive_threshold[%d]" % n, lambda o, n=n: pins.test_exhaustive_threshold(o, n)))
    for n in (4, 7, 9):
        out.append(("exhaustive_symmetric[%d]" % n, lambda o, n=n: pins.test_exhaustive_symmetric(o, n)))
    for name in ("exhaustive_ragged_tail", "looped_recurrence_all_thetas", "sorting_view", "library_reductions",
                 "monotone_and_sum_identity", "permutation_and_complement", "padding_rule",
                 "weights_by_replication", "cols_match_full", "golden_rle", "golden_allfill",
                 "rle_roundtrip_and_canonical", "rle_noncanonical_accepted", "rle_malformed_rejected",
                 "rle_encode_ignores_tail", "run_count", "count_against_numpy", "weighted_equals_replication"):
        out.append((name, getattr(pins, "test_" + name)))
    for n in (1, 3, 6, 10):
        out.append(("count_closed_form[%d]" % n, lambda o, n=n: pins.test_count_closed_form(o, n)))
    for w in ([1], [3, 1, 2], [5, 5, 1, 7, 2, 2], [1, 2, 4, 8, 16, 32, 64, 100]):
        out.append(("weighted_exhaustive%s" % w, lambda o, w=w: pins.test_weighted_exhaustive(o, w)))
    return out


def main(path):
    import oracle
    oracle.use_library(path)
    for name, fn in battery():
        try:
            fn(oracle)
        except Exception as e:  # noqa: BLE001  (any failure of a pin counts)
            print("pin failed: %s (%s: %s)" % (name, type(e).__name__, str(e)[:200]), flush=True)
            return 1
    print("all pins passed", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))

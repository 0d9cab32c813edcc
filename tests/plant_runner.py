"""Runs every oracle pin against one compiled oracle library (argv[1]).

Exit status 0 if all pins pass, 1 if any fails; prints the failing pins.
Used by test_oracle_plants.py in a child process, so a planted mistake that
crashes the library cannot take the test session down with it.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import pins  # noqa: E402


def main(path):
    orc = oracle.Oracle(path)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
    print("failed:", " ".join(failed) if failed else "none")
    return 1 if failed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))

"""Run the oracle pins against one built copy of the oracle library and print
the name of the first pin that fails (every failing pin with --all), one per
line (used by test_oracle_mutants)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import pins  # noqa: E402


def main(lib_path: str) -> None:
    orc = oracle.Oracle(lib_path)
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except Exception as exc:  # any failure of the pin counts
            print("FAILED", pin.__name__, type(exc).__name__, flush=True)
            if "--all" not in sys.argv:
                return  # one failing pin is enough to catch a mutant


if __name__ == "__main__":
    main(sys.argv[1])

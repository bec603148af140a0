"""`python -m paper_2309_14311_amd.traffic file.ini [--agent] [--stream] [--onestep]`:
the starter code's driver (`./traffic test.ini`) on the GPU, through the native
command-line program built next to the library."""
import os
import subprocess
import sys

CLI = os.path.join(os.path.dirname(os.path.abspath(__file__)), "nasch_traffic")


def main(argv=None) -> int:
    argv = sys.argv[1:] if argv is None else argv
    if not os.path.exists(CLI):
        print(f"{CLI} is not built; run python -m paper_2309_14311_amd.build", file=sys.stderr)
        return 2
    return subprocess.run([CLI, *argv]).returncode


if __name__ == "__main__":
    sys.exit(main())

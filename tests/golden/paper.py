"""Reader of the values the paper prints (fixtures in this folder)."""
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def iteration_counts():
    """{name: (grid side, iterations)} from paper_iteration_counts.txt."""
    out = {}
    with open(os.path.join(_HERE, "paper_iteration_counts.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            f = line.split()
            out[f[0]] = (int(f[1]), int(f[3]))
    return out


PAPER_250 = iteration_counts()["one_gpu_250"][1]
PAPER_1E9 = iteration_counts()["sixty_four_gpus_1e9"][1]

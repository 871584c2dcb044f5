"""The committed partition table of the autotuner (host only)."""
import pytest

from paper_1508_06103_amd import tune
from workloads.generate import BATCH_M, BATCH_N, class_instances


def test_table_covers_every_class_with_valid_partitions():
    tab = tune._load()["classes"]
    for n in BATCH_N:
        for M in BATCH_M:
            rec = tab[f"{n}x{M}"]
            parts, d = rec["parts"], rec["overlap"]
            assert len(parts) == 4 and all(p >= 1 for p in parts)
            assert all(p <= n + 1 for p in parts[:3]) and parts[3] <= M + 1
            assert d in tune.OVERLAPS
            # a candidate of the tuning mode that wrote the table (or its starting rule)
            if "tuning_batch" in tune._load():
                assert d == 1
                assert tuple(parts) in tune.mix_candidates(n, M) or tuple(parts) == tune.box_parts(n, M, 12)
                cap = tune._load().get("max_box_mb")
                if cap is not None:
                    assert tune.max_box_bytes(n, M, tuple(parts)) <= cap * 1e6
            else:
                assert (tuple(parts), d) in tune.candidates(n, M)


@pytest.mark.parametrize("n,M", [(8, 16), (20, 32), (24, 48)])
def test_parts_for_reads_the_class(n, M):
    prob = class_instances(n, M, count=1)[0]
    parts, d = tune.parts_for(prob)
    rec = tune._load()["classes"][f"{n}x{M}"]
    assert list(parts) == rec["parts"] and d == rec["overlap"]


@pytest.mark.parametrize("n,M", [(8, 24), (12, 32), (16, 16), (16, 48), (20, 16), (24, 48)])
def test_max_box_bytes_matches_the_partition(n, M):
    """The tuner's largest-box size equals the largest FP32 factor size over
    the boxes the partition really has (3 x 3 blocks of 4-byte values for
    every pair of box nodes at most one apart on every axis)."""
    from oracle.ras import subdomains

    class Mesh:
        nodes = (n + 1, n + 1, n + 1)

    Mesh.M = M
    for parts in tune.mix_candidates(n, M) + [tune.box_parts(n, M, 12)]:
        sizes = []
        for sd in subdomains(Mesh, parts, 1):
            b = 36
            for ext in sd.dims:
                b *= 3 * ext - 2
            sizes.append(b)
        assert tune.max_box_bytes(n, M, parts) == max(sizes)

"""Host-side checks of the serving runtime: configuration errors are reported
before any device work (no GPU needed)."""
import numpy as np
import pytest
import torch

from paper_2509_13300_amd import _lib as L


def genomes_view(n=3):
    g = L.ah_genomes()
    g.words = g.word_off = g.len = 0x1000  # never dereferenced: rejected first
    g.n = n
    g.max_len = 100
    return g


@pytest.mark.parametrize("cfg,match", [
    (dict(n_lanes=0), "n_lanes"), (dict(n_lanes=17), "n_lanes"), (dict(n_compilers=0), "n_compilers"),
    (dict(part_bases=0), "part_bases"), (dict(max_part_hits=0), "part_bases"),
    (dict(capacity_scale=-1.0), "capacity_scale"),
])
def test_bad_server_config_is_rejected(cfg, match):
    pool = torch.empty(1 << 16, dtype=torch.uint8)
    with pytest.raises(L.AhError, match=match) as e:
        L.ah_server_create(genomes_view(), np.ones(3, np.uint32), L.server_config(**cfg), pool)
    assert e.value.status == L.AH_ERR_INVALID_ARG


def test_tiny_pool_is_rejected():
    pool = torch.empty(1000, dtype=torch.uint8)
    with pytest.raises(L.AhError, match="pool") as e:
        L.ah_server_create(genomes_view(), np.ones(3, np.uint32), L.server_config(), pool)
    assert e.value.status == L.AH_ERR_INVALID_ARG

"""Host-side checks of the streaming call: argument validation and chunk
planning errors are reported before any device work (no GPU needed)."""
import numpy as np
import pytest
import torch

from paper_2509_13300_amd import _lib as L
from synth import plan


def host_collection(lengths):
    lengths = np.asarray(lengths, dtype=np.int64)
    off = L.ah_pack_layout(lengths)
    words = torch.zeros(2 * max(int(off[-1]), 1), dtype=torch.int32)
    return L.HostGenomes(words, off, lengths)


def call(hg, cfg, work_bytes=None, pairs=None):
    pairs = pairs or [plan.PairSpec("ACGTACGTACGT", "GGCCAATTGGCC", 1, 0, 50, 500)]
    need = L.ah_stream_workspace_bytes(hg, cfg, len(pairs), 64)
    work = torch.empty(need if work_bytes is None else work_bytes, dtype=torch.uint8)
    hits = torch.empty(64 * 16, dtype=torch.uint8)
    res = torch.empty(24, dtype=torch.uint8)
    amps = torch.empty(64 * 24, dtype=torch.uint8)
    ares = torch.empty(24, dtype=torch.uint8)
    L.ah_stream_query(hg, cfg, pairs, L.windows(pairs), L.tm_params(), hits, 64, res, amps, 64, ares,
                      work, stream=0)


def test_workspace_grows_with_slots_and_chunk():
    hg = host_collection([1000, 5000, 70000])
    a = L.ah_stream_workspace_bytes(hg, L.stream_config(4096, 2), 1, 1000)
    b = L.ah_stream_workspace_bytes(hg, L.stream_config(4096, 3), 1, 1000)
    c = L.ah_stream_workspace_bytes(hg, L.stream_config(8192, 3), 1, 1000)
    assert 0 < a < b < c
    assert b - a >= 4096 * 8  # one more slot of packed words
    assert L.ah_stream_workspace_bytes(hg, L.stream_config(4096, 1), 1, 1000) == 0


@pytest.mark.parametrize("chunk,slots,match", [
    (4096, 1, "n_slots"), (4096, 17, "n_slots"), (31, 2, "chunk_words"), (4097, 2, "chunk_words"),
])
def test_bad_config_is_rejected(chunk, slots, match):
    hg = host_collection([1000, 2000])
    with pytest.raises(L.AhError, match=match) as e:
        call(hg, L.stream_config(chunk, slots), work_bytes=1 << 20)
    assert e.value.status == L.AH_ERR_INVALID_ARG


def test_genome_larger_than_a_slot_is_a_limit_error():
    hg = host_collection([1000, 200000, 3000])  # 6250 + 32 words for the second
    cfg = L.stream_config(4096, 2)
    with pytest.raises(L.AhError, match="genome 1 spans") as e:
        call(hg, cfg)
    assert e.value.status == L.AH_ERR_LIMIT


def test_small_workspace_is_rejected():
    hg = host_collection([1000, 2000])
    cfg = L.stream_config(4096, 2)
    with pytest.raises(L.AhError, match="stream workspace") as e:
        call(hg, cfg, work_bytes=L.ah_stream_workspace_bytes(hg, cfg, 1, 64) - 1)
    assert e.value.status == L.AH_ERR_WORKSPACE


def test_bad_primer_is_rejected_before_device_work():
    hg = host_collection([1000])
    with pytest.raises(L.AhError) as e:
        call(hg, L.stream_config(4096, 2),
             pairs=[plan.PairSpec("ACGTUCGTACGT", "GGCCAATTGGCC", 1, 0, 50, 500)])
    assert e.value.status == L.AH_ERR_INVALID_PRIMER

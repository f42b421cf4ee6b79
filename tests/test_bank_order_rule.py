"""The stored order of the list chunks (the LDS-bank order that include/sindi.h states) as the
GPU tests check it: the helper's rule on hand-worked chunks, so that a wrong helper cannot
pass a wrong device layout."""
import numpy as np
import pytest

from parity import check_bank_order


def _one_list(docs_sorted, stored_docs, vals_sorted=None, stored_vals=None):
    """A one-tile, one-term index holding one list; raw slots padded to 4."""
    n = len(docs_sorted)
    groups = (n + 3) // 4
    pad = 4 * groups - n
    goff = np.zeros((1, 2), np.uint32)
    goff[0, 0] = np.uint32(pad) << np.uint32(30)
    goff[0, 1] = groups
    raw_doc = np.full(4 * groups, 4 * max(docs_sorted), np.uint16)
    raw_doc[:n] = 4 * np.asarray(stored_docs)
    if vals_sorted is None:
        vals_sorted = np.arange(1, n + 1, dtype=np.float32)
        pos = {d: i for i, d in enumerate(docs_sorted)}
        stored_vals = np.array([vals_sorted[pos[d]] for d in stored_docs], np.float32)
    raw_val = np.zeros(4 * groups, np.float32)
    raw_val[:n] = stored_vals
    raw = {"tile_doc": np.array([0, 20_000]), "tile_post": np.array([0, 4 * groups]),
           "term_goff": goff, "post_doc": raw_doc, "post_val": raw_val}
    ex = {"post_doc": np.asarray(docs_sorted, np.uint16), "post_val": vals_sorted}
    return raw, ex


def test_chunk_of_eight_fills_lanes_by_bank():
    # banks (document mod 32): 0, 32 and 64 share bank 0; 1 and 33 bank 1; 5, 7, 40 their own.
    docs = [0, 1, 5, 7, 32, 33, 40, 64]
    # (bank, document) order: 0, 32, 64, 1, 33, 5, 7, 40 -> slots 0, 1, 2, 3, 4, 5, 6, 7 (lanes
    # 0 and 1 of one half: slot 4 r + p for r = 0, 1)
    stored = [0, 32, 64, 1, 33, 5, 7, 40]
    check_bank_order(*_one_list(docs, stored))
    with pytest.raises(AssertionError):
        check_bank_order(*_one_list(docs, docs))  # ascending is not the stored rule here


def test_chunk_of_four_or_fewer_stays_ascending():
    docs = [3, 35, 67, 99]  # one bank: a one-group chunk keeps its order
    check_bank_order(*_one_list(docs, docs))
    with pytest.raises(AssertionError):
        check_bank_order(*_one_list(docs, [3, 67, 35, 99]))


def test_full_chunk_spreads_a_bank_over_instructions_and_half_waves():
    # 256 documents, eight per bank: the rule gives every (instruction, half-wave) pass one
    # posting of each bank, so no pass has two postings in one bank
    docs = sorted(range(0, 256 * 3, 3))
    order = sorted(docs, key=lambda d: (d % 32, d))
    slots = [4 * (32 * h + r) + p for r in range(32) for h in range(2) for p in range(4)]
    stored = [0] * 256
    for k, s in enumerate(slots):
        stored[s] = order[k]
    check_bank_order(*_one_list(docs, stored))
    st = np.array(stored).reshape(64, 4)  # [lane, instruction]
    for p in range(4):
        for h in range(2):
            banks = st[32 * h:32 * h + 32, p] % 32
            assert len(set(banks.tolist())) == 32

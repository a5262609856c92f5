"""RANLUX-form state export/import and value-granular skip, against the
oracle (section 2: the final engine stores the 24 RANLUX numbers and the
carry; seeding/skipping, section 2.4)."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx
from rlx_util import ints_to_words, records_to_tensor, tensor_to_records, words_to_ints

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_export_matches_oracle():
    rng = random.Random(1)
    xs = [0, 1, O.M - 1, 2 ** 336, 2 ** 336 - 1] + [rng.randrange(O.M) for _ in range(500)]
    recs = [(x, rng.randrange(12), 404) for x in xs]
    st = records_to_tensor(recs)
    packed, carry, pos = rlx.export_ranlux(st)
    pk = words_to_ints(packed.cpu().numpy())
    for (x, ps, _), d, c, q in zip(recs, pk, carry.cpu().tolist(), pos.cpu().tolist()):
        nums, cc = O.to_ranlux(x)
        assert d == O.RANLUX.pack(nums) and c == cc and q == ps


def test_import_round_trip_and_generation():
    rng = random.Random(2)
    p = 218
    recs = [(O.seed(i, p), rng.randrange(12), p) for i in range(300)]
    st = records_to_tensor(recs)
    packed, carry, pos = rlx.export_ranlux(st)
    st2 = rlx.new_states(len(recs))
    rlx.check_errors()
    rlx.import_ranlux(st2, packed, carry, p, pos=pos)
    assert rlx.check_errors() == 0
    assert torch.equal(st2, st)


def test_import_rejects_degenerate_and_noncanonical():
    p = 24
    g = O.RANLUX
    rng = random.Random(3)
    # all numbers 2^24 - 1 with carry 1 maps to X = m (= 0 mod m)
    degenerate = (1 << 576) - 1
    cases = [(degenerate, 1)]
    # non-canonical SWB states: random numbers and carry whose LCG form does
    # not convert back to them
    while len(cases) < 40:
        d, c = rng.getrandbits(576), rng.randrange(2)
        x = g.to_lcg(d, c)
        if x >= O.M or g.to_ranlux(x) != (d, c):
            cases.append((d, c))
    n = len(cases)
    st = records_to_tensor([(5, 0, p)] * n)
    before = st.clone()
    packed = torch.from_numpy(ints_to_words([d for d, _ in cases])).to(DEV)
    carry = torch.tensor([c for _, c in cases], dtype=torch.int32, device=DEV)
    rlx.check_errors()
    rlx.import_ranlux(st, packed, carry, p)
    assert rlx.check_errors() == 0x8
    assert torch.equal(st, before)
    # after 24 SWB steps every state is canonical and imports; its values
    # continue the SWB sequence
    stepped = [g.swb_steps(d, c, 24) for d, c in cases[1:]]
    packed = torch.from_numpy(ints_to_words([d for d, _ in stepped])).to(DEV)
    carry = torch.tensor([c for _, c in stepped], dtype=torch.int32, device=DEV)
    st = rlx.new_states(len(stepped))
    rlx.import_ranlux(st, packed, carry, p)
    assert rlx.check_errors() == 0
    out = rlx.generate_u64(st, 36, p).cpu().numpy()
    for (d, c), row in zip(stepped, out):
        exp = []
        dd, cc = d, c
        for _ in range(3):
            nums = g.digits(dd)
            exp += [nums[2 * k] | (nums[2 * k + 1] << 24) for k in range(12)]
            dd, cc = g.swb_steps(dd, cc, p)
        assert row.tolist() == exp


def test_skip_values_equals_drawing():
    rng = random.Random(4)
    p = 2048
    n = 300
    recs = [(O.seed(i + 1, p), rng.randrange(12), p) for i in range(n)]
    vs = [0, 1, 11, 12, 13, 2 ** 64 - 1, 2 ** 63 + 7] + [rng.getrandbits(rng.randrange(1, 65)) for _ in range(n - 7)]
    st = records_to_tensor(recs)
    vt = torch.from_numpy(np.array(vs, dtype=np.uint64).view(np.int64)).to(DEV)
    rlx.skip_values(st, vt, p)
    got = tensor_to_records(st)
    for (x, pos, _), v, g in zip(recs, vs, got):
        steps, newpos = divmod(pos + v, 12)
        assert g == (O.skip(x, steps, p), newpos, p)
    # small skips equal drawing the values
    st1 = records_to_tensor(recs[:50])
    st2 = st1.clone()
    rlx.skip_values(st1, 29, p)
    rlx.generate_u64(st2, 29, p)
    assert torch.equal(st1, st2)


def test_import_checks_tensor_shapes():
    st = rlx.new_states(4)
    packed = torch.zeros((4, 9), dtype=torch.int64, device=DEV)
    carry = torch.zeros(4, dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError):
        rlx.import_ranlux(st, packed[:3], carry, 24)
    with pytest.raises(ValueError):
        rlx.import_ranlux(st, packed, carry.to(torch.int64), 24)
    with pytest.raises(ValueError):
        rlx.import_ranlux(st, packed, carry, 24, pos=torch.zeros(5, dtype=torch.int32, device=DEV))

"""Statistical smoke checks of the GPU output (not pins: the values are
pinned bit for bit against the oracle elsewhere; these only catch gross
damage such as repeated or zeroed blocks in a large launch).  The paper's
quality claim rests on TestU01 BigCrush (section 2.5), which is not run
here."""
import numpy as np
import pytest
import scipy.stats
import torch

import paper_2106_02504_amd as rlx

pytestmark = pytest.mark.gpu


def test_uniform_doubles_smoke():
    p, n, count = 2048, 4096, 4096          # 2^24 doubles
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=1)          # id 0 starts from X = 1
    u = rlx.generate_f64(st, count, p).view(-1)
    N = u.numel()
    mean = float(u.mean())
    var = float(u.var())
    assert abs(mean - 0.5) < 6 * (1 / 12 / N) ** 0.5
    assert abs(var - 1 / 12) < 6 * (1 / 180 / N) ** 0.5
    bins = 1024
    counts = torch.bincount((u * bins).to(torch.int64), minlength=bins).cpu().numpy()
    chi2 = float(((counts - N / bins) ** 2 / (N / bins)).sum())
    assert scipy.stats.chi2.sf(chi2, bins - 1) > 1e-6
    # each of the 48 bits of the values is set about half the time
    v = (u * 2.0 ** 48).to(torch.int64)
    for bit in (0, 1, 23, 24, 46, 47):
        ones = int(((v >> bit) & 1).sum())
        assert abs(ones - N / 2) < 6 * (N / 4) ** 0.5, bit


def test_float32_smoke():
    p, n, count = 404, 2048, 8192
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=7)
    f = rlx.generate_f32(st, count, p).view(-1).to(torch.float64)
    N = f.numel()
    assert abs(float(f.mean()) - 0.5) < 6 * (1 / 12 / N) ** 0.5
    counts = torch.bincount((f * 256).to(torch.int64), minlength=256).cpu().numpy()
    chi2 = float(((counts - N / 256) ** 2 / (N / 256)).sum())
    assert scipy.stats.chi2.sf(chi2, 255) > 1e-6

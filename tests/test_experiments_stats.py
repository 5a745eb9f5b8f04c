"""The experiment statistics (pruning curve, recall, errors) on hand-made
outputs whose values are worked out by hand; CPU tensors, no GPU."""
import torch

import paper_1110_1328_amd as P
from paper_1110_1328_amd import experiments as E


def test_pruning_curve_by_hand():
    # 6 candidates, k = 32, 4 levels: decided at levels 0, 0, 1, 3, 3, 2
    code = torch.tensor([0 << 6 | 0, 1 << 6 | 0, 0 << 6 | 1, 2 << 6 | 3, 0 << 6 | 3, 1 << 6 | 2], dtype=torch.uint8)
    curve = E.pruning_curve(code, 32, 4)
    assert curve == [(32, 4 / 6), (64, 3 / 6), (96, 2 / 6), (128, 0.0)]


def test_quality_by_hand():
    # truth for 5 candidates; positives at t = 0.7: candidates 0, 2, 3
    truth = torch.tensor([0.9, 0.2, 0.7, 0.75, 0.69], dtype=torch.float64)
    res = P.make_result(5, 8, device="cpu")
    res.acc_idx[:3] = torch.tensor([3, 0, 4], dtype=torch.int64).view(torch.uint64)
    res.acc_val[:3] = torch.tensor([0.80, 0.90, 0.60])
    res.n_accepted[0] = 3
    mask, idx, val = E.accepted_mask(res, 5)
    assert mask.tolist() == [True, False, False, True, True]
    q = E.quality(mask, idx, val, truth, 0.7)
    assert q["positives"] == 3 and q["accepted"] == 3 and q["accepted_positives"] == 2
    assert abs(q["recall"] - 2 / 3) < 1e-12
    assert q["false_positives"] == 1
    # errors: |0.80 - 0.75| = 0.05, |0.90 - 0.90| = 0, |0.60 - 0.69| = 0.09 (fp32 values)
    errs = [abs(float(torch.tensor(0.80, dtype=torch.float32)) - 0.75), abs(float(torch.tensor(0.90, dtype=torch.float32)) - 0.9),
            abs(float(torch.tensor(0.60, dtype=torch.float32)) - 0.69)]
    assert abs(q["mean_error"] - sum(errs) / 3) < 1e-12
    assert abs(q["max_error"] - max(errs)) < 1e-12
    assert abs(q["frac_error_gt"] - sum(e > 0.05 for e in errs) / 3) < 1e-12


def test_truncated_list_rejected():
    res = P.make_result(5, 2, device="cpu")
    res.n_accepted[0] = 3
    try:
        E.accepted_mask(res, 5)
    except ValueError:
        return
    raise AssertionError("a truncated list must not be scored")

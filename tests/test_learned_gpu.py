"""The learned start end to end on the GPU: training with the library's own
kernels lowers the loss, and the shipped network (trained on multipliers the
plain loop settled to) reaches the plain loop's best feasible profit in fewer
samples on held-out instances."""
import os

import numpy as np
import pytest

from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import learn as L

pytestmark = pytest.mark.gpu


def test_training_lowers_the_loss(need_gpu):
    import torch
    # sixteen QKP members (index % 4 in {0, 1}): one set each, so that random
    # targets can be fitted set by set
    ms = [L.learn_instance(50_000 + 4 * (i // 2) + i % 2) for i in range(16)]
    pk = B.pbit_net_pack([p for p, _ in ms], [q for _, q in ms])
    d = L.Trainer.upload(pk)
    y = torch.from_numpy(np.random.default_rng(0).uniform(0.8, 1.2, pk["sets"]).astype(np.float32)).cuda()
    T = L.Trainer(seed=3)
    losses = []
    for _ in range(300):
        T.train_step(d, y, 3e-3)
        losses.append(float(T.loss.cpu()[0]))
    assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])


@pytest.mark.skipif(not os.path.exists(L.DEFAULT_WEIGHTS), reason="no trained weights shipped")
def test_learned_start_needs_fewer_samples(need_gpu):
    """Held-out QKP instances (Table 1's settings): the shipped network's start
    reaches the plain loop's best in far fewer samples than lambda_0 = 0, and is
    on a par with the scale-only start (the analytic scale times the training
    targets' median).  Beating that constant is not asserted: on 500 held-out
    QKP instances the network's margin over it is 5-11 % in geometric mean with
    95 % intervals that include no gain."""
    count, K = 48, 150
    ms = [L.learn_instance(L.EVAL_SEED_BASE + 7000 + 4 * (i // 2) + i % 2) for i in range(count)]
    probs, pars = [p for p, _ in ms], [q for _, q in ms]
    lam0 = L.predict_lambda0(probs, pars).cpu().numpy().reshape(count, 32)
    lam_c = L.scale_only_lambda0(probs, pars)
    plain = L.run_loop(probs, pars, K)
    learned = L.run_loop(probs, pars, K, lambda0=lam0)
    const = L.run_loop(probs, pars, K, lambda0=lam_c)
    res = L.compare(plain, learned, K, pars[0].replicas)
    res_c = L.compare(plain, const, K, pars[0].replicas)
    print(res, res_c, flush=True)
    # the plain loop needs many rounds before its multipliers make samples
    # feasible; the learned start has feasible samples at least as often
    assert learned["has"][-1].sum() >= plain["has"][-1].sum()
    assert res["plain_feasible"] >= 6
    assert res["reached_target"] >= res["plain_feasible"] - 1
    assert res["geomean_ratio_plain_over_other"] > 2.0
    # not behind the scale-only start by more than a quarter
    assert res["geomean_ratio_plain_over_other"] > 0.75 * res_c["geomean_ratio_plain_over_other"]

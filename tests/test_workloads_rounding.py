"""The input-rounding helpers shared by the tests: FP16 / BF16 rounding of the MLP
weights (the values a reduced-precision MLP multiplies) and the weight mask of the
packed MLP."""
import numpy as np
import torch

import workloads as wl


def test_round_bf16_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(wl.round_bf16(a), ref)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even neighbour (1)
    one = np.float32(1.0)
    assert wl.round_bf16(np.array([one + np.float32(2.0 ** -8)]))[0] == 1.0
    assert wl.round_bf16(np.array([one + np.float32(3 * 2.0 ** -8)]))[0] == np.float32(1 + 2.0 ** -6)


def test_mlp_weight_mask_and_rounding():
    for n_in, hidden, layers in ((10, 16, 1), (13, 32, 2)):
        n = wl.mlp_size(n_in, hidden, wl.N_OUT, layers)
        mask = wl.mlp_weight_mask(n_in, hidden, layers)
        assert mask.size == n
        n_bias = hidden * layers + wl.N_OUT
        assert (~mask).sum() == n_bias
        m = wl.xavier_uniform_mlp(np.random.default_rng(1), n_in, hidden, wl.N_OUT, layers)
        m[~mask] = 0.123456789  # biases stay FP32
        r = wl.round_mlp_weights(m, n_in, hidden, layers, "f16")
        np.testing.assert_array_equal(r[~mask], m[~mask])
        np.testing.assert_array_equal(r[mask], m[mask].astype(np.float16).astype(np.float32))
        r = wl.round_mlp_weights(m, n_in, hidden, layers, "bf16")
        np.testing.assert_array_equal(r[mask], wl.round_bf16(m[mask]))

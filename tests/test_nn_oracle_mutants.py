"""The surrogate oracle's pins have teeth: plausible mistakes planted in a
copy of oracle/nn_oracle.py (on the CPU only) must each make at least one of
its pins fail."""
from __future__ import annotations

import os
import types

import pytest
import torch

from oracle import nn_oracle
from tests import test_nn_oracle_pins as pins

SRC = os.path.join(os.path.dirname(nn_oracle.__file__), "nn_oracle.py")

MUTANTS = {
    # both decay rates exchanged: step 1 is unchanged, step 2 is not
    # the two decay rates exchanged everywhere (moments and bias corrections):
    # steps with m_hat = g and v_hat = g^2 are unchanged, the second step of
    # gradients (1, 0) is not
    "adam_betas_swapped": (('    """Bias-corrected Adam; returns new (w, m, v)."""\n',
                            '    """Bias-corrected Adam; returns new (w, m, v)."""\n    b1, b2 = b2, b1\n'),),
    # only the moment updates exchanged
    "adam_moment_rates_swapped": (("    m = b1 * m + (1 - b1) * g\n    v = b2 * v + (1 - b2) * g * g\n",
                                   "    m = b2 * m + (1 - b2) * g\n    v = b1 * v + (1 - b1) * g * g\n"),),
    "adam_no_bias_correction_of_v": (("    vh = v / (1 - b2 ** step)\n", "    vh = v\n"),),
    "adam_bias_power_off_by_one": (("    mh = m / (1 - b1 ** step)\n", "    mh = m / (1 - b1 ** (step + 1))\n"),),
    "adam_no_sqrt": (("np.sqrt(vh) + eps", "vh + eps"),),
    "adam_eps_inside_sqrt": (("np.sqrt(vh) + eps", "np.sqrt(vh + eps)"),),
    "conv_taps_transposed": (("wk = w.reshape(cout, ks, ks, cin).permute(0, 3, 1, 2)\n    y = ",
                              "wk = w.reshape(cout, ks, ks, cin).permute(0, 3, 2, 1)\n    y = "),),
    "conv_kernel_flipped": (("y = _nhwc(F.conv2d(_nchw(x), wk, bias, padding=ks // 2))",
                             "y = _nhwc(F.conv2d(_nchw(x), wk.flip(2, 3), bias, padding=ks // 2))"),),
    "pool_sums": (("return _nhwc(F.avg_pool2d(_nchw(x), 2))", "return _nhwc(4 * F.avg_pool2d(_nchw(x), 2))"),),
    "skip_not_concatenated": (("        h = torch.cat([up2(q(h)), skips[lvl]], dim=-1)\n",
                               "        h = torch.cat([up2(q(h)), 0 * skips[lvl]], dim=-1)\n"),),
    "stored_mask_of_input": (("        g = back(f\"d{lvl}b\", s(g * (b > 0)), a)\n",
                              "        g = back(f\"d{lvl}b\", s(g * (a > 0)), a)\n"),),
    "stored_skip_gradient_dropped": (("            g = _pool2_adjoint(gx) + skip_g[lvl - 1]\n",
                                      "            g = _pool2_adjoint(gx)\n"),),
}

def load_mutant(name: str) -> types.ModuleType:
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"mutation anchor of {name} not unique: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType(f"nn_oracle_{name}")
    exec(compile(src, f"<{name}>", "exec"), mod.__dict__)
    return mod


def run_pins(O) -> list[str]:
    """Names of the pins that fail for oracle module O."""
    failed = []
    checks = {f.__name__: f for f in pins.ADAM_PINS}
    checks["conv_direct_loops"] = lambda O: pins.check_conv_direct_loops(O, 3)
    checks["pool_upsample"] = pins.check_pool_and_upsample
    checks["finite_differences"] = pins.check_unet_finite_differences
    checks["stored_identity"] = pins.check_stored_backward_identity
    for name, f in checks.items():
        try:
            f(O)
        except AssertionError:
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_every_pin():
    assert run_pins(nn_oracle) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(name):
    torch.manual_seed(0)
    assert run_pins(load_mutant(name)), f"mutant {name} passes every pin"


def test_fully_swapped_decay_rates_pass_the_first_step_and_fail_the_second():
    """The mistake that step 1 cannot see is caught by the two-step closed form."""
    failed = run_pins(load_mutant("adam_betas_swapped"))
    assert "pin_adam_first_step" not in failed and "pin_adam_constant_gradient" not in failed
    assert "pin_adam_second_step_separates_the_decay_rates" in failed

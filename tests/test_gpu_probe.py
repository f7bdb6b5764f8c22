"""The issue-rate probe (kde_issue_rates): the per-clock rates behind the pair
kernels' roofline, measured on the part with the library's own code.

The published FP32 vector peak of the part is 128 FP32 lanes of add/mul/fma
per clock and CU, reached with packed (two-wide) instructions; the library is
built without them, and unpacked instructions retire half that rate.
v_exp_f32 retires 32 lanes per clock and CU.  These tests check that the
measured rates are consistent with that model: unpacked plain FP32 near 64
lanes, exp2 near 32, neither above its assumed figure by more than noise, and
the LSCV term mix (one mul, one exp2, one add, one fma) not faster than the
sequential-issue bound at the packed rate."""
import pytest

pytestmark = pytest.mark.gpu

VALU, TRANS = 128.0, 32.0
UNPACKED = 64.0
MIX_BOUND = 1.0 / (3.0 / VALU + 1.0 / TRANS)  # terms per clock per CU


@pytest.fixture(scope="module")
def rates():
    import paper_1505_01998_amd as kde

    with kde.Context(0) as c:
        r = c.issue_rates()
    print({k: round(v, 2) if isinstance(v, float) else v for k, v in r.items()})
    return r


def test_device_shape(rates):
    assert rates["cus"] >= 1 and rates["clock_hz"] > 1e8


def test_plain_and_exp_rates_within_assumed_unit_counts(rates):
    for k in ("add_f32", "mul_f32", "fma_f32"):
        assert 0.8 * UNPACKED < rates[k] <= 1.03 * UNPACKED, (k, rates[k])
    assert 0.8 * TRANS < rates["exp_f32"] <= 1.03 * TRANS, rates["exp_f32"]


def test_lscv_mix_below_sequential_issue_bound(rates):
    assert 0.0 < rates["lscv_mix"] <= 1.03 * MIX_BOUND, rates["lscv_mix"]
    assert 0.0 < rates["lscv_mix_zero"] <= 1.03 * MIX_BOUND, rates["lscv_mix_zero"]


def test_probe_rejects_null(rates):
    import ctypes

    import paper_1505_01998_amd as kde

    with kde.Context(0) as c:
        assert kde.lib.kde_issue_rates(c.ctx, None) == kde.KDE_E_INVAL
    assert kde.lib.kde_issue_rates(None, ctypes.byref(kde.kde_issue_info())) == kde.KDE_E_INVAL

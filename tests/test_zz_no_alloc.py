"""amg_level_features_noalloc (the entry point for callers that cannot
allocate) against amg_level_features through the C ABI: every level of two
hierarchies, called back to back, the second hierarchy smaller, so the
second call runs on the scratch array the first one left behind."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1503_01287_amd as amg  # noqa: E402

DEV = torch.device("cuda:0")


def _compare(s):
    for l in range(s.num_levels):
        want = s.level_features(l)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device=DEV)
        s.level_features_noalloc(l, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got)), (l, got)
        assert np.allclose(got, want, rtol=1e-14, atol=0.0), (l, got, want)


def test_noalloc_features_match_two_calls_second_smaller():
    big = amg.AMGSolver(amg.problems.elasticity(8), smoother="JA-1-1-0.5")
    small = amg.AMGSolver(amg.problems.laplace(3), smoother="JA-1-1-0.5")
    assert big.level_info(0).n_lin + big.level_info(0).n_quad > small.level_info(0).n_lin + small.level_info(0).n_quad
    _compare(big)
    _compare(small)
    # and the large one again after the small one
    _compare(big)
    big.close()
    small.close()


def test_noalloc_features_on_a_side_stream():
    s = amg.AMGSolver(amg.problems.elasticity(5), smoother="JA-1-1-0.5")
    want = s.level_features(0)
    st = torch.cuda.Stream()
    out = torch.zeros(8, dtype=torch.float64, device=DEV)
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        s._stream = st
        s.level_features_noalloc(0, out)
    st.synchronize()
    s._stream = None
    assert np.allclose(out.cpu().numpy(), want, rtol=1e-14, atol=0.0)
    s.close()

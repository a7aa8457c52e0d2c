"""The Python binding refuses, before any library call, tensors whose shape,
dtype or device does not match what the call reads or writes (a wrong-sized
output would otherwise be written past its end)."""
import pytest

from helpers import api

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    return api()


def test_outputs_of_the_wrong_shape_or_device_are_refused(A):
    s = A.System("lorenz", 3, [10.0, 28.0, 8 / 3])
    x = torch.zeros((3, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError, match="hist must have shape"):
        A.project_histogram(s, x, 0, 1, (0.0, 1.0), (0.0, 1.0), 8, 8,
                            hist=torch.zeros((4, 4), dtype=torch.int32, device="cuda:0"))
    with pytest.raises(ValueError, match="n_dropped"):
        A.project_histogram(s, x, 0, 1, (0.0, 1.0), (0.0, 1.0), 8, 8,
                            n_dropped=torch.zeros(1, dtype=torch.int32, device="cuda:0"))
    eye = [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]
    with pytest.raises(ValueError, match="img must have shape"):
        A.render_image(s, x, (0, 1, 2), eye, 8, 8, img=torch.zeros((8, 8), dtype=torch.int32, device="cuda:0"))
    with pytest.raises(ValueError, match="GPU tensor"):
        A.render_image(s, x, (0, 1, 2), eye, 8, 8, img=torch.zeros((8, 8, 3), dtype=torch.int32))
    with pytest.raises(ValueError, match="GPU tensor"):
        A.integrate(s, x, 0.01, 10, pparams=torch.ones((1, 64), dtype=torch.float64), pp_slot=[1])
    ws = torch.empty(A.adjoint_workspace_size(s, x, 10, 5), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ValueError, match="lam must have shape"):
        A.adjoint(s, x, 0.01, 10, 5, ws, torch.zeros((3, 32), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError, match="mu is given"):
        A.adjoint(s, x, 0.01, 10, 5, ws, torch.zeros_like(x), mu=torch.zeros((1, 64), dtype=torch.float64,
                                                                                 device="cuda:0"))
    with pytest.raises(ValueError, match="mu_global needs"):
        A.adjoint(s, x, 0.01, 10, 5, ws, torch.zeros_like(x),
                  mu_global=torch.zeros(2, dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()

"""The GEMM accuracy experiments of Sec. IV-A (Figs. 2-4) on the GPU: mean
relative Frobenius error against the FP64 product over seeded 256 x 256
operands, for uniform [-1, 1], maximal-exponent and Gaussian-exponent inputs.
The GPU's mean errors agree with the oracle's on the same operands, and they
show the paper's orderings: on [-1, 1] x3 > FP32 > x6 >= x9 (Fig. 2); with a
wide exponent range the FP32 GEMM and x6 are nearly identical (Figs. 3, 4)."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu

N, SEEDS = 256, 20
GENS = {
    "uniform": lambda shape, sd: workloads.uniform(shape, sd),
    "max_exp": lambda shape, sd: workloads.max_exp(shape, sd, K=N),
    "gauss_exp": lambda shape, sd: workloads.gauss_exp(shape, sd),
}


def _mean_errors(bfx, orc, gen):
    gpu, ora = {}, {}
    tC = torch.empty((N, N), dtype=torch.float32, device="cuda")
    for sd in range(SEEDS):
        A, B = gen((N, N), 3000 + 2 * sd), gen((N, N), 3001 + 2 * sd)
        Z = A.astype(np.float64) @ B.astype(np.float64)
        zn = np.linalg.norm(Z)
        tA, tB = dev(A), dev(B)
        for v in (3, 6, 9, 0):
            if v:
                bfx.gemm(v, tA, tB, tC)
                Co = orc.gemm(v, A, B)
            else:
                bfx.sgemm_fp32(tA, tB, tC)
                Co = orc.sgemm(A, B)
            C = tC.cpu().numpy().astype(np.float64)
            gpu.setdefault(v, []).append(np.linalg.norm(C - Z) / zn)
            ora.setdefault(v, []).append(np.linalg.norm(Co.astype(np.float64) - Z) / zn)
    return ({v: float(np.mean(e)) for v, e in gpu.items()}, {v: float(np.mean(e)) for v, e in ora.items()})


@pytest.mark.parametrize("name", list(GENS))
def test_figures_2_to_4_orderings(bfx, orc, name):
    g, o = _mean_errors(bfx, orc, GENS[name])
    for v in g:
        assert abs(g[v] - o[v]) <= 0.2 * o[v], (name, v, g[v], o[v])
    assert g[3] > 10 * max(g[6], g[0])
    if name == "uniform":
        assert g[3] > g[0] > 2 * g[6] and g[6] >= 0.99 * g[9], g
    else:
        assert 0.7 < g[6] / g[0] < 1.4, g

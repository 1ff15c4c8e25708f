"""The five workload configurations (sizes, seeds, budgets) of the benchmark.

The paper's workload (Sec. IV-E) is the Cascadia data-space matrix with 600
candidate sensors, N_t = 420 observations each and a budget of 175; it is not
available, so seeded synthetic K of the same candidate count and budget stand
in for it (see ``synth``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Spec:
    name: str
    N_s: int
    N_t: int
    n_m: int
    seed: int
    budget: int
    c: float = 0.01
    precision: str = "fp64"          # "fp64" | "mixed_f32" | "mixed_bf16x3"
    k_dtype: str = "f64"             # dtype K is formed and handed over in
    notes: str = ""

    @property
    def N_d(self) -> int:
        return self.N_s * self.N_t


CONFIGS = {
    "small_fp64_64x16": Spec("small_fp64_64x16", 64, 16, 4096, 0, 16, precision="fp64"),
    "fp64_600x128": Spec("fp64_600x128", 600, 128, 76800, 1, 175, precision="fp64",
                         notes="oracle on a 100-sensor subsample"),
    "mixed_600x128": Spec("mixed_600x128", 600, 128, 76800, 1, 175, precision="mixed_f32",
                          notes="same K as fp64_600x128; R in FP32"),
    "large_1500x96": Spec("large_1500x96", 1500, 96, 40000, 2, 175, precision="mixed_f32",
                          k_dtype="f32"),
    # the paper's shape: K (252,000^2) is never whole on the GPU; F (40 GB FP32) stays resident and
    # K's row panels are formed one GEMM at a time and packed into the working copy (135 GB FP32)
    "paper_600x420": Spec("paper_600x420", 600, 420, 40000, 3, 175, precision="mixed_f32", k_dtype="f32",
                          notes="F resident, K formed and packed by row panels"),
}


def batched_instance_specs(n: int = 48):
    """The uneven batched designs: instance i draws its shape from seed 100+i.

    N_s uniform in [40, 400], N_t from {16, 32, 64}, noise factor c log-uniform
    in [1e-3, 1e-1], n_m = 2 N_d, budget = N_s // 4, F seed 100+i.
    """
    out = []
    for i in range(n):
        rng = np.random.default_rng(100 + i)
        N_s = int(rng.integers(40, 401))
        N_t = int(rng.choice([16, 32, 64]))
        c = float(10.0 ** rng.uniform(-3.0, -1.0))
        out.append(Spec(f"batched_{i}", N_s, N_t, 2 * N_s * N_t, 100 + i, N_s // 4, c=c,
                        precision="mixed_f32", k_dtype="f32"))
    return out

"""The five benchmark workloads: codes, error rates, shot counts, variants.

Discounts alpha of Momentum-BP and EWAInit-BP follow the paper's selection
rule (ten evenly spaced values in [0, 1], the best one kept: section IV-A,
applied in section IV-B with one value for all code lengths), evaluated on the
FP64 oracle by ``tests/golden/choose_alpha.py``; its output
``tests/golden/alpha_choice.json`` holds the scores and a CPU test checks that
the values below equal its choices.  AdaGrad-BP uses alpha = 5 and Momentum-BP
gamma = 0 (section IV-A).
"""

ADAGRAD_ALPHA = 5.0
MOMENTUM_GAMMA = 0.0

# configuration 1: planar d=3, depolarizing p = 0.05, 10^4 shots, iter_max 50, BP and EWAInit
CONFIG1 = dict(family="planar", size=3, p=0.05, shots=10000, max_iter=50)
# configuration 2: toric L=8, p swept 0.02..0.16 in 8 steps, 2^20 shots per p, iter_max 100,
# Momentum-BP, AdaGrad-BP, EWAInit-BP
CONFIG2 = dict(family="toric", size=8, p=(0.02, 0.04, 0.06, 0.08, 0.10, 0.12, 0.14, 0.16), shots=1 << 20,
               max_iter=100)
# configuration 3: the mixed batch; (family, size, shot multiplier of 2^18)
CONFIG3_CODES = (("planar", 5, 1), ("planar", 7, 1), ("planar", 9, 2), ("planar", 11, 4), ("planar", 13, 4),
                 ("toric", 6, 1), ("toric", 10, 2), ("toric", 14, 4),
                 ("xzzx", 5, 1), ("xzzx", 9, 2), ("xzzx", 13, 4))
CONFIG3 = dict(p=0.08, base_shots=1 << 18, max_iter=100)
# configuration 5: large codes, messages in HBM
CONFIG5_CODES = (("planar", 31), ("toric", 32))
CONFIG5 = dict(p=0.10, shots=1 << 18, max_iter=200)

# chosen discounts per (configuration, variant)
ALPHA = {
    (1, "ewainit"): 0.6,
    (2, "momentum"): 0.9,
    (2, "ewainit"): 0.7,
    (3, "ewainit"): 0.6,
    (5, "ewainit"): 0.6,
}


def alpha(config: int, variant: str) -> float:
    """Discount of `variant` in configuration `config` (AdaGrad: its step rate; BP: 1)."""
    if variant == "adagrad":
        return ADAGRAD_ALPHA
    if variant == "bp":
        return 1.0
    a = ALPHA[(config, variant)]
    if a is None:
        raise KeyError(f"no discount chosen for configuration {config}, {variant}")
    return a

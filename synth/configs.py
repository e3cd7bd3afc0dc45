"""The five workload configurations and their seeds.

Seeds per configuration k: map 1000+k, views 2000+k, edits 3000+k,
arrivals 4000+k (PCG64 via numpy.random.default_rng).
"""

SEEDS = {
    k: {"map": 1000 + k, "views": 2000 + k, "edits": 3000 + k,
        "arrivals": 4000 + k}
    for k in range(1, 6)
}

# Map shapes and terrain statistics.  "dual" is the share of cells that carry
# an upper slab; 0.109 is the double-level share of the paper's level
# (Section 2).  Blob sizes are cells per connected slab blob.
CONFIGS = {
    1: dict(name="c1-plain-256", W=256, H=256, dual=0.20, period=64,
            cliffs="steps", n_cliffs=6, blob=(8, 200)),
    2: dict(name="c2-plain-2048", W=2048, H=2048, dual=0.30, period=256,
            cliffs="terraces", n_cliffs=16, blob=(8, 200)),
    3: dict(name="c3-edits-2048x16384", W=2048, H=16384, dual=0.109,
            period=256, cliffs="terraces", n_cliffs=96, blob=(8, 200)),
    4: dict(name="c4-batched-2048x16384", W=2048, H=16384, dual=0.109,
            period=256, cliffs="terraces", n_cliffs=96, blob=(8, 200)),
    5: dict(name="c5-served-2048x16384", W=2048, H=16384, dual=0.109,
            period=256, cliffs="terraces", n_cliffs=96, blob=(8, 200)),
}


def config(k):
    c = dict(CONFIGS[k])
    c["k"] = k
    c["seeds"] = SEEDS[k]
    return c

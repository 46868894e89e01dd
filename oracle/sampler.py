"""Oracle of the hyper-reduction sample-point selection (Section 3.2.1).

TEST INFRASTRUCTURE ONLY.

The paper draws the sample material points by plain stochastic sampling and
redraws them at every time step; it does not fix the distribution.  Reading
used here (and on the GPU, from the same published definitions, written
independently): stratified sampling without replacement -- the reference
particle index range [0, P) is cut into S strata [floor(kP/S),
floor((k+1)P/S)), and stratum k contributes index lo_k + (u_k mod len_k), with
u_k a 64-bit counter-based random number.

u_k comes from the SplitMix64 output function of Steele, Lea and Flood,
"Fast splittable pseudorandom number generators" (OOPSLA 2014), as published
by Vigna:  mix(c) = fin(c + 0x9E3779B97F4A7C15) with
fin(z) = z3 ^ (z3 >> 31), z3 = (z2 ^ (z2 >> 27)) * 0x94D049BB133111EB,
z2 = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 (all mod 2^64), chained as
    key  = mix(mix(mix(seed) ^ instance) ^ step),   u_k = mix(key ^ k).
Pure Python integers, so there is no rounding anywhere.
"""
MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix(c):
    z = (c + GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def stream_key(seed, instance, step):
    return mix(mix(mix(seed & MASK) ^ (instance & MASK)) ^ (step & MASK))


def stratified_samples(seed, instance, step, n_samples, n_particles):
    """Sample indices (ascending, distinct) for one instance and time step."""
    if n_samples <= 0 or n_samples > n_particles:
        raise ValueError("need 0 < n_samples <= n_particles")
    key = stream_key(seed, instance, step)
    out = []
    for k in range(n_samples):
        lo = (k * n_particles) // n_samples
        hi = ((k + 1) * n_particles) // n_samples
        u = mix(key ^ k)
        out.append(lo + u % (hi - lo))
    return out

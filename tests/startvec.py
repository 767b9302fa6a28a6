"""Start vector of the library's ||A||_2 power method, written on the test
side from the published definition of the splitmix64 generator (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014; the
finalizer constants of Stafford's "Mix13" variant used by Java's
SplittableRandom and by Vigna's splitmix64.c): for index i the state is
seed + i + 0x9E3779B97F4A7C15, mixed by z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31, and the top 53 bits
map to [-1, 1).  The oracle's power method takes this vector as its start,
so that its estimate and the library's follow the same iteration."""
import numpy as np

SEED = 0x5EED


def splitmix_raw(idx, seed: int = SEED) -> np.ndarray:
    """64-bit outputs for the states seed + i + 0x9E3779B97F4A7C15."""
    with np.errstate(over="ignore"):
        z = np.asarray(idx, dtype=np.uint64) + np.uint64(seed) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix_start(n: int, seed: int = SEED) -> np.ndarray:
    z = splitmix_raw(np.arange(n, dtype=np.uint64), seed)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0

"""Plain oracle of the keyframe-list optimisation schedule (GSFusion Sec. III-B-3 and the
implementation details of Sec. IV-A).

TEST INFRASTRUCTURE ONLY: the product library never imports or calls anything here.
It shares no code with the library's schedule.

At each time step the seeding of the new frame reports how many Gaussians it added.  The
paper takes that number as the frame's information gain:

* a frame whose count exceeds the keyframe threshold (50 in the experiments) is a
  keyframe: it joins the keyframe list and is optimised for m iterations;
* any other frame is optimised for n iterations, and the remaining m - n iterations go
  to keyframes drawn at random from the list: the first m - n of the list after a
  shuffle.

Readings where the paper is silent (each is stated here and in the library header):

* one iteration optimises one view (one forward, loss and backward, one optimiser step);
  the frame's own iterations come first, then one iteration per drawn keyframe in the
  shuffled order;
* "exceeds" is strict (count > threshold); a negative threshold makes every frame a
  keyframe;
* with ``store_all`` (the ScanNet++ setting, where every frame is kept in the list) every
  frame joins the list while m or n still follows the threshold, so the random
  iterations happen on the non-keyframes; a frame joins the list after its own draw, so
  it is never drawn at its own time step;
* a list shorter than m - n gives each of its keyframes one iteration;
* the shuffle: keyframe i of the list (0-based, in insertion order) gets the key
  h(h(seed, frame + 1), i + 1), where h(s, k) is the k-th output of the SplitMix64
  generator seeded with s (Steele, Lea and Flood, 2014: add k times the golden-ratio
  increment 0x9E3779B97F4A7C15 to s, then apply its 64-bit mixing function); the list is
  ordered by (key, i) ascending.  The generator is counter based, so every side that
  follows this definition draws the same keyframes.
"""
from __future__ import annotations

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def mix64(z: int) -> int:
    """SplitMix64's output function (variant 13 of Stafford's mixers)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64(seed: int, k: int) -> int:
    """The k-th output (k >= 1) of SplitMix64 seeded with `seed`."""
    return mix64((seed + k * GAMMA) & MASK)


def shuffled(keyframes, seed: int, frame: int):
    """The keyframe list in its shuffled order for time step `frame`."""
    s = splitmix64(seed, frame + 1)
    keyed = [(splitmix64(s, i + 1), i, kf) for i, kf in enumerate(keyframes)]
    keyed.sort()
    return [kf for _, _, kf in keyed]


class Schedule:
    def __init__(self, m: int, n: int, threshold: int, store_all: bool = False, seed: int = 0):
        assert 0 <= n <= m
        self.m, self.n, self.threshold = m, n, threshold
        self.store_all, self.seed = bool(store_all), seed & MASK
        self.keyframes: list[int] = []

    def step(self, frame: int, new_gaussians: int):
        """(is_keyframe, frames optimised by this time step's iterations, in order)."""
        is_kf = new_gaussians > self.threshold
        if is_kf:
            self.keyframes.append(frame)
            return True, [frame] * self.m
        iters = [frame] * self.n
        iters += shuffled(self.keyframes, self.seed, frame)[: self.m - self.n]
        if self.store_all:
            self.keyframes.append(frame)
        return False, iters

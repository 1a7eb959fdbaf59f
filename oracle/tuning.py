"""Amortization model of dynamic autotuning (oracle; test infrastructure only).

Sect. 5.4 ("Dynamic tuning of the benchmark set") models the cost of tuning
at run time.  With s tuning steps whose kernels take t_avg on average and
n - s further invocations of a well-performing kernel taking t_well:

* relative performance (Eq. 3) compares running n invocations with the
  well-performing kernel from the start against tuning first.  The equation
  as printed is the ratio of the tuned run's time to the untuned run's time
  (>= 1), while the text calls rp a performance fraction (rp = 0.9 is 90 %);
  the reading that is consistent with Eq. 4 and with the worked example is
  the inverse ratio, rp = n t_well / (s t_avg + (n - s) t_well);
* invocations needed for a target rp (Eq. 4):
  n = rp s (t_avg / t_well - 1) / (1 - rp);
* random-search steps to find one of a fraction r of well-performing
  configurations with probability p (Eq. 5): s = log_{1-r}(1 - p).
"""
from __future__ import annotations

import math


def relative_performance(n: float, s: float, t_avg: float, t_well: float) -> float:
    return n * t_well / (s * t_avg + (n - s) * t_well)


def invocations(rp: float, s: float, t_avg: float, t_well: float) -> float:
    if not (0.0 < rp < 1.0) or t_well <= 0:
        raise ValueError("need 0 < rp < 1 and t_well > 0")
    return rp * s * (t_avg / t_well - 1.0) / (1.0 - rp)


def steps(r: float, p: float) -> float:
    if not (0.0 < r < 1.0) or not (0.0 <= p < 1.0):
        raise ValueError("need 0 < r < 1 and 0 <= p < 1")
    return math.log(1.0 - p) / math.log(1.0 - r)

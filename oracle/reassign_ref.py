"""Reassignment of under-used components (Alg. 1, `reassign`; Sec. 3.1). Test infrastructure only.

Plain NumPy restatement of the step that precedes `fit` in each frame: sample n points biased
towards a low per-point evidence bound, pick the n least-used components, and move the means of
those components onto the sampled points. Readings (the paper leaves them open):
- per-point bound: the point's log normaliser LSE_n (nats) of the last E-step;
- biased sampling: Gumbel-top-n with logits -LSE_n, i.e. sampling n points without replacement
  with probabilities proportional to exp(-LSE_n); the Gumbel noise g_n = -ln(-ln u_n) is an input;
- least used: smallest posterior alpha_k;
- order keys: a value is compared through the order-preserving 64-bit image of its FP64 bits with
  the low 25 bits replaced by the index (so values equal to about 2^-27 relative tie, and ties go
  to the lower index);
- the i-th sampled point (largest key first) goes to the i-th component (least used first); the
  new mean is written into both the frame prior and the posterior, nothing else changes.
"""
import numpy as np

IDX_BITS = 25
IDX_MASK = np.uint64((1 << IDX_BITS) - 1)


def ord64(x):
    """Order-preserving map of float64 values onto uint64 (x < y  <=>  ord64(x) < ord64(y))."""
    b = np.ascontiguousarray(np.asarray(x, np.float64)).view(np.uint64)
    neg = (b >> np.uint64(63)) == np.uint64(1)
    return np.where(neg, ~b, b | np.uint64(1 << 63))


def index_keys(values, descending):
    """Sort keys: the order image of each value (complemented for descending order) with the low
    IDX_BITS bits replaced by the element's index."""
    v = np.asarray(values, np.float64)
    o = ord64(v)
    if descending:
        o = ~o
    idx = np.arange(v.size, dtype=np.uint64)
    return (o & ~IDX_MASK) | idx


def select(values, n, descending):
    """Indices of the n smallest keys (see index_keys), in key order."""
    keys = index_keys(values, descending)
    order = np.sort(keys)[:n]
    return (order & IDX_MASK).astype(np.int64)


def reassign(X, lse, gumbel, alpha, n):
    """Returns (points, comps): point points[i] becomes the new mean of component comps[i]."""
    N, K = len(lse), len(alpha)
    if n < 0 or n > min(N, K):
        raise ValueError("n must be in 0..min(N, K)")
    pts = select(np.asarray(gumbel, np.float64) - np.asarray(lse, np.float64), n, descending=True)
    comps = select(alpha, n, descending=False)
    return pts, comps


def apply(m_prior, m_post, X, pts, comps):
    """New means: both records of component comps[i] take the coordinates of point pts[i]."""
    mp, mq = np.array(m_prior, np.float64), np.array(m_post, np.float64)
    xs = np.asarray(X, np.float32).astype(np.float64)
    mp[comps] = xs[pts]
    mq[comps] = xs[pts]
    return mp, mq

"""Leaf jobs of the recursion tree, counted from the oracle's splits (test
infrastructure): the leaves the library hands to its leaf kernels, i.e. all
leaves except the sparse and with-replacement ones of at most INLINE_MAX
values, which its tree kernels sample themselves; constant leaves (a range
of one element, with replacement) count one job per 2^16 values."""
INLINE_MAX = 32
FILL_PIECE = 1 << 16
LEAF_RANGE = 1 << 32


def jobs(ref, variant, n, N, seed, n0=4096, dense_ratio=16):
    count, todo = 0, [(1, N, n)]
    while todo:
        node, Nv, nv = todo.pop()
        if nv == 0:
            continue
        if variant == 1 and Nv == 1:
            count += -(-nv // FILL_PIECE)
            continue
        if nv < n0 and Nv <= LEAF_RANGE:
            if variant == 1:
                inline = nv <= INLINE_MAX
            else:
                inline = nv <= INLINE_MAX and dense_ratio * nv < Nv
            count += 0 if inline else 1
            continue
        l = Nv // 2
        L = ref.binom(nv, l, Nv, seed, node) if variant else ref.hyp(nv, l, Nv, seed, node)
        todo.append((2 * node, l, L))
        todo.append((2 * node + 1, Nv - l, nv - L))
    return count

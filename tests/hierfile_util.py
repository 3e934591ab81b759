"""Hierarchy-file helpers for the tests: rewrite a current file in the first
format version (which had no fused restrictions)."""


def fnv1a(b):
    h = 1469598103934665603
    for c in b:
        h = ((h ^ c) * 1099511628211) & (2 ** 64 - 1)
    return h


def to_version_1(data: bytes) -> bytes:
    """Rewrite a version-2 hierarchy file as version 1: the same fields
    without each level's fused restriction."""
    out = bytearray()
    pos = 0

    def take(n):
        nonlocal pos
        out.extend(data[pos:pos + n])
        pos += n

    def skip_vec(item):
        nonlocal pos
        n = int.from_bytes(data[pos:pos + 8], "little", signed=True)
        pos += 8 + n * item

    def take_vec(item):
        n = int.from_bytes(data[pos:pos + 8], "little", signed=True)
        take(8 + n * item)

    def take_csr():
        take(8)
        take_vec(4), take_vec(4), take_vec(8)

    def skip_csr():
        nonlocal pos
        pos += 8
        skip_vec(4), skip_vec(4), skip_vec(8)

    assert int.from_bytes(data[8:12], "little") == 2
    take(8)
    out.extend((1).to_bytes(4, "little"))
    pos += 4
    take(8 + 3 * 4 + 3 * 4 + 2)  # AMG options, n, n_o, n_g, two flags
    take_vec(4)  # permutation
    for _ in range(6):
        take_csr()
    for _ in range(2):  # the two hierarchies
        nl = int.from_bytes(data[pos:pos + 4], "little", signed=True)
        take(4 + 1)
        take_vec(8)
        for _ in range(nl):
            take_csr(), take_csr(), take_csr()  # A, P, R
            skip_csr()  # fused restriction
            take_vec(8), take_vec(4)  # l1 norms, aggregates
    assert pos == len(data) - 8
    return bytes(out) + fnv1a(bytes(out)).to_bytes(8, "little")

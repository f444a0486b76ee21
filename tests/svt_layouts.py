"""Row lengths that select each Jacobi layout with single floats per lane.

A row of nr floats is nr4 = ceil(nr / 4) float4 chunks.  With two-row
blocks of 8 or 16 lanes, nch = nr4 // lanes whole chunks per lane (1 to 3)
plus a remainder of 4 (nr4 - nch lanes) floats held as ceil(rem / lanes)
single floats per lane, when that is at most 2.  Each entry is
(lanes per pair, chunks per lane, single floats per lane, row length); the
row lengths are not multiples of 4 where possible, so the zero padding of
the last chunk is exercised too."""

TAIL_LAYOUTS = [
    (8, 1, 1, 35), (8, 1, 2, 43), (8, 2, 1, 66), (8, 2, 2, 75), (8, 3, 1, 99), (8, 3, 2, 106),
    (16, 1, 1, 71), (16, 1, 2, 87), (16, 2, 1, 130), (16, 2, 2, 150), (16, 3, 1, 195), (16, 3, 2, 214),
]

// Host-side ghost rules: where the value of a ghost-extended cell comes
// from.  The same rules as value_i / value_ij of the device code (two ghost
// layers per side; the i sides are resolved first, the j sides apply their
// rule to the i-resolved rows, which defines the corner ghosts).  Used to build the
// per-tile halo source tables of the fused kernel and the inverse ghost map
// of the adjoint.
#include "hb_internal.hpp"

namespace hb {

GSrc ghost_src_i(const std::vector<BlockDesc> &B, int b, int i, int j) {
    const BlockDesc &K = B[b];
    if (i >= 0 && i < K.ni) return GSrc{1, b, i, j, 0};
    const int side = i < 0 ? 0 : 1;
    const int k = i < 0 ? -1 - i : i - K.ni;
    switch (K.bc[side]) {
        case HB_BC_PERIODIC: return GSrc{1, b, i < 0 ? i + K.ni : i - K.ni, j, 0};
        case HB_BC_WALL: return GSrc{1, b, side == 0 ? k : K.ni - 1 - k, j, 1};
        case HB_BC_CUT: {
            const int a = K.cut_blk[side];
            return GSrc{1, a, side == 0 ? B[a].ni - 1 - k : k, j, 0};
        }
        default: return GSrc{0, b, 0, 0, 0};
    }
}

GSrc ghost_src(const std::vector<BlockDesc> &B, int b, int i, int j) {
    const BlockDesc &K = B[b];
    if (j >= 0 && j < K.nj) return ghost_src_i(B, b, i, j);
    const int side = j < 0 ? 2 : 3;
    const int k = j < 0 ? -1 - j : j - K.nj;
    GSrc s;
    switch (K.bc[side]) {
        case HB_BC_PERIODIC: return ghost_src_i(B, b, i, j < 0 ? j + K.nj : j - K.nj);
        case HB_BC_WALL:
            s = ghost_src_i(B, b, i, side == 2 ? k : K.nj - 1 - k);
            s.mir ^= 1;
            return s;
        case HB_BC_WAKECUT:
            if (i < K.wake || i >= K.ni - K.wake) return ghost_src_i(B, b, K.ni - 1 - i, k);
            s = ghost_src_i(B, b, i, k);
            s.mir ^= 1;
            return s;
        case HB_BC_CUT: {
            const int a = K.cut_blk[side];
            return ghost_src_i(B, a, i, side == 2 ? B[a].nj - 1 - k : k);
        }
        default: return GSrc{0, b, 0, 0, 0};
    }
}

// Moving no-slip wall image (ghost (i, j) of block b on a rigidly moving
// grid): the node index (within the block's node arrays) of the first node
// of the wall face whose midpoint velocity the image takes, and the block
// owning it; {-1, ..} when the ghost is no wall image.  The same column
// rule as the plain kernels' wall_image_motion: a ghost column takes its
// i-periodic partner column, the glued block's column across an i cut, else
// the nearest column.
WallFace wall_face(const std::vector<BlockDesc> &B, int b, int i, int j) {
    const BlockDesc &K = B[b];
    int side;
    if (j < 0) side = 2;
    else if (j >= K.nj) side = 3;
    else return WallFace{-1, 0};
    const int kind = K.bc[side];
    if (!(kind == HB_BC_WALL || (kind == HB_BC_WAKECUT && side == 2))) return WallFace{-1, 0};
    if (kind == HB_BC_WAKECUT && (i < K.wake || i >= K.ni - K.wake)) return WallFace{-1, 0};
    int col = i, src = b;
    if (i < 0) {
        if (K.bc[0] == HB_BC_PERIODIC) col = i + K.ni;
        else if (K.bc[0] == HB_BC_CUT) src = K.cut_blk[0], col = B[src].ni + i;
        else col = 0;
    } else if (i >= K.ni) {
        if (K.bc[1] == HB_BC_PERIODIC) col = i - K.ni;
        else if (K.bc[1] == HB_BC_CUT) src = K.cut_blk[1], col = i - K.ni;
        else col = K.ni - 1;
    }
    const BlockDesc &S = B[src];
    return WallFace{(int64_t)(side == 2 ? 0 : S.nj) * (S.ni + 1) + col, src};
}

}  // namespace hb

// Host-side ghost rules: where the value of a ghost-extended cell comes
// from.  The same rules as value_ij of the device code (two ghost layers
// per side; the i sides are resolved first, then the j sides, which
// defines the corner ghosts; across a cut the partner block's own rules
// apply to what is still outside it).  Used to build the per-tile halo
// source tables of the fused kernel and the inverse ghost map of the
// adjoint.
#include "hb_internal.hpp"

namespace hb {

GSrc ghost_src(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S, int b, int i, int j,
               int *wall) {
    int mir = 0;
    // the last wall face mirrored at: block, side, position along the side
    auto seen = [&](int side, int p) {
        if (wall) {
            wall[0] = b;
            wall[1] = side;
            wall[2] = p;
        }
    };
    if (wall) wall[0] = -1;
    for (int hop = 0; hop < kGhostHops; ++hop) {
        const BlockDesc &K = B[b];
        if (i < 0 || i >= K.ni) {
            const int side = i < 0 ? 0 : 1;
            const int k = i < 0 ? -1 - i : i - K.ni;
            switch (K.bc[side]) {
                case HB_BC_PERIODIC: i = i < 0 ? i + K.ni : i - K.ni; break;
                case HB_BC_WALL: seen(side, j); i = side == 0 ? k : K.ni - 1 - k; mir ^= 1; break;
                case HB_BC_CUT: {
                    if (!glued_at(K, S.data(), side, j)) {
                        if (K.rest[side] != HB_BC_WALL) return GSrc{0, b, 0, 0, mir};
                        seen(side, j);
                        i = side == 0 ? k : K.ni - 1 - k;
                        mir ^= 1;
                        break;
                    }
                    int a, ia, ja;
                    cut_cell(B.data(), S.data(), b, side, k, j, &a, &ia, &ja);
                    b = a; i = ia; j = ja;
                    break;
                }
                default: return GSrc{0, b, 0, 0, mir};
            }
            continue;
        }
        if (j < 0 || j >= K.nj) {
            const int side = j < 0 ? 2 : 3;
            const int k = j < 0 ? -1 - j : j - K.nj;
            switch (K.bc[side]) {
                case HB_BC_PERIODIC: j = j < 0 ? j + K.nj : j - K.nj; break;
                case HB_BC_WALL: seen(side, i); j = side == 2 ? k : K.nj - 1 - k; mir ^= 1; break;
                case HB_BC_WAKECUT:
                    if (i < K.wake || i >= K.ni - K.wake) {
                        i = K.ni - 1 - i;
                        j = k;
                    } else {
                        seen(side, i);
                        j = k;
                        mir ^= 1;
                    }
                    break;
                case HB_BC_CUT: {
                    if (!glued_at(K, S.data(), side, i)) {
                        if (K.rest[side] != HB_BC_WALL) return GSrc{0, b, 0, 0, mir};
                        seen(side, i);
                        j = side == 2 ? k : K.nj - 1 - k;
                        mir ^= 1;
                        break;
                    }
                    int a, ia, ja;
                    cut_cell(B.data(), S.data(), b, side, k, i, &a, &ia, &ja);
                    b = a; i = ia; j = ja;
                    break;
                }
                default: return GSrc{0, b, 0, 0, mir};
            }
            continue;
        }
        return GSrc{1, b, i, j, mir};
    }
    return GSrc{-1, b, 0, 0, mir};     // did not end (refused at grid creation)
}

bool ghosts_resolve(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S) {
    for (int b = 0; b < (int)B.size(); ++b)
        for (int j = -2; j < B[b].nj + 2; ++j)
            for (int i = -2; i < B[b].ni + 2; ++i) {
                if (i >= 0 && i < B[b].ni && j >= 0 && j < B[b].nj) continue;
                if (ghost_src(B, S, b, i, j).cell < 0) return false;
            }
    return true;
}

// Moving no-slip wall image (ghost (i, j) of block b on a rigidly moving
// grid): the node index (within the block's node arrays) of the first node
// of the wall face whose midpoint velocity the image takes, and the block
// owning it; {-1, ..} when the ghost is no wall image.  The face is the one
// at which the ghost's resolution mirrors (the rule of the plain kernels'
// wall_image_face); walls lie on j sides only (hb_set_motion).
WallFace wall_face(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S, int b, int i, int j) {
    int w[3];
    ghost_src(B, S, b, i, j, w);
    if (w[0] < 0 || w[1] < 2) return WallFace{-1, 0};
    const BlockDesc &K = B[w[0]];
    return WallFace{(int64_t)(w[1] == 2 ? 0 : K.nj) * (K.ni + 1) + w[2], w[0]};
}

}  // namespace hb

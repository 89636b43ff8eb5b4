// Host build of the device DEMAP routines, so that the CPU test-suite can
// check the exact child order (Sec. III-A-2) exhaustively without a GPU.
#include "vp_device.hpp"

extern "C" {

// tier 0: rank 0 only; tier 1: ranks 0..1; tier 2: ranks 0..2; tier 3: any
// rank (table lookup); tier 4: the region-table DEMAP (any rank).  The routines take the centre c and cp = c - 1/2,
// formed here in float32 from the given centres.
int vp_host_demap(const float *cx, const float *cy, const int32_t *rank, int n, int tier, float *a,
                  float *b) {
    for (int k = 0; k < n; ++k) {
        const float cpx = cx[k] - 0.5f, cpy = cy[k] - 0.5f;
        float aa, bb;
        if (tier == 0) {
            if (rank[k] != 0) return -1;
            vp_demap0(cpx, cpy, aa, bb);
        } else if (tier == 1) {
            if (rank[k] > 1) return -1;
            vp_demap1(cpx, cpy, cx[k], cy[k], rank[k], aa, bb);
        } else if (tier == 2) {
            if (rank[k] > 2) return -1;
            vp_demap2(cpx, cpy, cx[k], cy[k], rank[k], aa, bb);
        } else if (tier == 3) {
            vp_demapN(cpx, cpy, cx[k], cy[k], rank[k], VP_DEMAP_LUT, aa, bb);
        } else {
            vp_demap_region(cpx, cpy, cx[k], cy[k], rank[k], VP_REGION_LUT, aa, bb);
        }
        a[k] = aa;
        b[k] = bb;
    }
    return 0;
}
}

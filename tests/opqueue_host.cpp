// Host-side check of the bound on queued bitmap switches (built and run by
// tests/test_opqueue_host.py with hipcc, host code only; no GPU is touched).
// Replays on a host OpQueue the largest sequence of switches one release of
// slots can queue - the re-activation of a full block, a rollback for every
// failed invalidation attempt but the last, and the three switches of the
// successful invalidation - and then one push too many.
#include <cstdio>

#include "../paper_1908_05845_amd/csrc/smmo_device.hpp"

int main()
{
    using namespace smmo;
    OpQueue q;
    q.reset();
    int n = 0;
    bool ok = q.push(bm_active(0), 7, +1);
    ++n;
    for (int a = 0; a + 1 < kInvalidateAttempts; ++a, ++n) ok = q.push(bm_active(0), 7, -1) && ok;
    ok = q.push(bm_active(0), 7, -1) && ok;
    ok = q.push(bm_alloc(0), 7, -1) && ok;
    ok = q.push(BM_FREE, 7, +1) && ok;
    n += 3;
    std::printf("worst_case_pushes %d max_ops %d max_release_ops %d accepted %d overflow %d\n", n, kMaxOps,
                kMaxReleaseOps, ok ? 1 : 0, q.overflow ? 1 : 0);
    const bool extra = q.push(BM_FREE, 8, +1);
    std::printf("extra_push_accepted %d overflow %d pending %d\n", extra ? 1 : 0, q.overflow ? 1 : 0,
                q.pending() ? 1 : 0);
    return 0;
}

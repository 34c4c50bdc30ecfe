// Drives the serving engine's host-only admission rule and arena
// (paper_cs_0308004_amd/csrc/admission.h) through fixed scenarios and prints
// one line per check: "ok <name>" or "FAIL <name>".  Built and run by
// tests/test_serve_admission.py with the host compiler; needs no GPU.
#include <cstdio>
#include <vector>

#include "admission.h"

using namespace dpg;

static int failures = 0;
static void check(bool ok, const char *name) {
    std::printf("%s %s\n", ok ? "ok" : "FAIL", name);
    if (!ok) ++failures;
}

int main() {
    const size_t A = 256;
    {
        // arena of 64 KiB with 3 slot workspaces of 5000 B kept by the server
        Arena a(65536, A);
        size_t off;
        for (int i = 0; i < 3; ++i) a.alloc(5000, &off);
        const size_t capacity = a.size() - a.in_use();
        check(capacity == 65536 - 3 * 5120, "capacity is the arena less the rounded slot blocks");
        // a request between the capacity and the arena size fails at once
        AdmitResult r = admit_head(a, capacity, 60000, 0, false);
        check(r.kind == ADMIT_FAIL && a.in_use() == 3 * 5120, "request above capacity fails, arena untouched");
        // rounding counts: output and workspace of capacity / 2 + 1 each
        r = admit_head(a, capacity, capacity / 2 + 1, capacity / 2 + 1, false);
        check(r.kind == ADMIT_FAIL, "rounded output + workspace above capacity fails");
        // exactly the capacity fits
        r = admit_head(a, capacity, capacity - 1024, 1000, false);
        check(r.kind == ADMIT_OK && r.has_out && r.has_ws && a.in_use() == a.size(), "request of exactly the capacity");
        // with the arena full the next request waits, or fails when nothing will free memory
        AdmitResult w = admit_head(a, capacity, 256, 0, false);
        check(w.kind == ADMIT_WAIT, "full arena: wait");
        w = admit_head(a, capacity, 256, 0, true);
        check(w.kind == ADMIT_FAIL && a.in_use() == a.size(), "full arena while stopping: fail");
        // releasing makes room again
        a.release(r.out_off);
        a.release(r.ws_off);
        w = admit_head(a, capacity, 256, 512, false);
        check(w.kind == ADMIT_OK && w.has_out && w.has_ws, "admitted after release");
    }
    {
        // fragmentation: 4 blocks of 16 KiB, free the 1st and 3rd; 24 KiB
        // fits the capacity but no hole: wait, and a failed workspace
        // reservation gives the output block back
        Arena a(65536, A);
        size_t o[4];
        for (int i = 0; i < 4; ++i) a.alloc(16384, &o[i]);
        a.release(o[0]);
        a.release(o[2]);
        AdmitResult r = admit_head(a, a.size(), 24576, 0, false);
        check(r.kind == ADMIT_WAIT && a.in_use() == 32768, "fragmented arena: wait, nothing reserved");
        r = admit_head(a, a.size(), 16384, 16384 + 1, false);
        check(r.kind == ADMIT_WAIT && a.in_use() == 32768 && a.free_blocks() == 2,
              "workspace does not fit: output block returned");
        r = admit_head(a, a.size(), 16384, 16384, false);
        check(r.kind == ADMIT_OK && a.in_use() == 65536, "both holes used");
    }
    {
        // zero-byte requests need no block
        Arena a(1024, A);
        AdmitResult r = admit_head(a, 1024, 0, 0, false);
        check(r.kind == ADMIT_OK && !r.has_out && !r.has_ws && a.in_use() == 0, "empty request");
    }
    {
        // a queue served in order: admitted while they fit, then the head waits
        Arena a(4096, A);
        std::vector<size_t> reqs = {1000, 1000, 1000, 1000, 1000};
        std::vector<AdmitResult> got;
        for (size_t b : reqs) {
            AdmitResult r = admit_head(a, a.size(), b, 0, false);
            if (r.kind != ADMIT_OK) break;
            got.push_back(r);
        }
        check(got.size() == 4 && a.in_use() == 4096, "head-of-line: four of five admitted");
        a.release(got[1].out_off);
        AdmitResult r = admit_head(a, a.size(), 1000, 0, false);
        check(r.kind == ADMIT_OK && r.out_off == got[1].out_off, "fifth takes the freed block");
    }
    {
        // launch selection: the head decides; batched requests are taken in
        // order past unbatched ones, up to the batch limit
        using V = std::vector<bool>;
        check(select_launch(V{}, 8).empty(), "empty queue: nothing to launch");
        std::vector<size_t> t = select_launch(V{false, true, true}, 8);
        check(t.size() == 1 && t[0] == 0, "unbatched head runs alone");
        t = select_launch(V{true, false, true, true, false, true}, 8);
        check(t == std::vector<size_t>({0, 2, 3, 5}), "batched requests taken past unbatched ones");
        t = select_launch(V{true, true, true, true, true}, 3);
        check(t == std::vector<size_t>({0, 1, 2}), "batch limit");
        t = select_launch(V{true, true, true}, 1);
        check(t.size() == 1 && t[0] == 0, "per-request mode takes the head only");
    }
    return failures ? 1 : 0;
}

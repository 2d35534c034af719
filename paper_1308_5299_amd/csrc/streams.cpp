// Fork/join of independent work onto pooled streams (grouped entry points).
//
// Work items that touch the same grid (the grid's transform workspaces) share
// one stream, in call order; other items get their own, up to the pool size.
// Every pooled stream first waits on an event recorded on the caller's
// stream, and the caller's stream finally waits on every pooled stream, so the
// grouped call is stream-ordered like the single ones.  Streams are created
// once per device at the default priority and kept until the process ends.
#include <map>
#include <vector>

#include "mlcr_internal.h"

namespace mlcr {

static constexpr int kPoolStreams = 8;

static int pool_streams(std::vector<hipStream_t> **out) {
    static std::map<int, std::vector<hipStream_t>> pools;
    int dev = 0;
    MLCR_HIP_CHECK(hipGetDevice(&dev));
    std::vector<hipStream_t> &p = pools[dev];
    while ((int)p.size() < kPoolStreams) {
        hipStream_t st;
        MLCR_HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        p.push_back(st);
    }
    *out = &p;
    return MLCR_OK;
}

int StreamFork::begin(hipStream_t parent_, const std::vector<const void *> &keys) {
    parent = parent_;
    std::vector<hipStream_t> *pool;
    int rc;
    if ((rc = pool_streams(&pool))) return rc;
    std::map<const void *, int> slot;
    item_stream.resize(keys.size());
    for (size_t i = 0; i < keys.size(); i++) {
        auto it = slot.find(keys[i]);
        int k;
        if (it != slot.end()) {
            k = it->second;
        } else {
            k = (int)slot.size() % kPoolStreams;
            slot[keys[i]] = k;
        }
        item_stream[i] = (*pool)[k];
    }
    for (hipStream_t st : item_stream) {
        bool seen = false;
        for (hipStream_t u : used) seen = seen || u == st;
        if (!seen) used.push_back(st);
    }
    hipEvent_t ev;
    MLCR_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    MLCR_HIP_CHECK(hipEventRecord(ev, parent));
    for (hipStream_t st : used) MLCR_HIP_CHECK(hipStreamWaitEvent(st, ev, 0));
    MLCR_HIP_CHECK(hipEventDestroy(ev));
    return MLCR_OK;
}

int StreamFork::join() {
    for (hipStream_t st : used) {
        hipEvent_t ev;
        MLCR_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        MLCR_HIP_CHECK(hipEventRecord(ev, st));
        MLCR_HIP_CHECK(hipStreamWaitEvent(parent, ev, 0));
        MLCR_HIP_CHECK(hipEventDestroy(ev));
    }
    used.clear();
    return MLCR_OK;
}

}  // namespace mlcr

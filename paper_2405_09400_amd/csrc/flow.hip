// Flow update (work in progress).
#include "ctx.hpp"

struct FlowState {};

void flow_release(dd_ctx* c) {
    delete c->flow;
    c->flow = nullptr;
}

extern "C" dd_status flow_update(dd_ctx* c, dd_flow_stats*) {
    if (c) c->err = "flow_update: not built yet";
    return DD_ESTATE;
}

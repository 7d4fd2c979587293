// serve.cpp -- placeholder, replaced by the serving loop.
#include "mfgemm.h"
extern "C" int mfg_server_create(const mfg_server_config*, mfg_server**) { return MFG_ERR_UNSUPPORTED; }
extern "C" int mfg_submit(mfg_server*, const mfg_request*, uint64_t*) { return MFG_ERR_UNSUPPORTED; }
extern "C" int mfg_poll(mfg_server*, uint64_t, mfg_result*) { return MFG_ERR_UNSUPPORTED; }
extern "C" int mfg_server_drain(mfg_server*) { return MFG_ERR_UNSUPPORTED; }
extern "C" int mfg_server_get_stats(mfg_server*, mfg_server_stats*) { return MFG_ERR_UNSUPPORTED; }
extern "C" int mfg_server_destroy(mfg_server*) { return MFG_ERR_UNSUPPORTED; }

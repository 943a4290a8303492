// The operator entry points of the C ABI: argument checks, then launches.
#include <cmath>
#include <cstdint>

#include "internal.h"

using namespace rt;

namespace {

int check_dev_ptr(const void *ptr, size_t n, const char *name)
{
    if (n == 0) return RT_OK;
    if (!ptr) return fail(RT_E_ARG, "%s is NULL", name);
    if ((uintptr_t)ptr % 16 != 0) return fail(RT_E_ARG, "%s is not 16-byte aligned", name);
    return RT_OK;
}

int check_device(const Plan &p)
{
    int dev = -1;
    RT_HIP(hipGetDevice(&dev));
    if (dev != p.device)
        return fail(RT_E_ARG, "current device %d is not the plan's device %d", dev, p.device);
    return RT_OK;
}

int prologue(const rt_plan *plan)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    return check_device(plan->impl);
}

}  // namespace

extern "C" int rt_forward(const rt_plan *plan, const float *f, float *g, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if ((rc = check_dev_ptr(f, nf_of(p.g), "f"))) return rc;
    if ((rc = check_dev_ptr(g, ng_of(p.g), "g"))) return rc;
    return launch_forward(p, f, g, CONTRACT_STORE, nullptr, nullptr, 0.f, nullptr,
                             (hipStream_t)stream);
}

extern "C" int rt_adjoint(const rt_plan *plan, const float *g, float *f_out, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if ((rc = check_dev_ptr(g, ng_of(p.g), "g"))) return rc;
    if ((rc = check_dev_ptr(f_out, nf_of(p.g), "f_out"))) return rc;
    return launch_adjoint(p, g, f_out, (hipStream_t)stream);
}

extern "C" int tv_grad(const rt_plan *plan, const float *f, float lambda2, float *pout, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if (!std::isfinite(lambda2)) return fail(RT_E_ARG, "lambda2 is not finite");
    if ((rc = check_dev_ptr(f, nf_of(p.g), "f"))) return rc;
    if ((rc = check_dev_ptr(pout, 4 * n4_of(p.g), "p"))) return rc;
    return launch_tv_grad(p, f, lambda2, pout, (hipStream_t)stream);
}

extern "C" int tv_div(const rt_plan *plan, const float *pin, float lambda2, float *f_out, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if (!std::isfinite(lambda2)) return fail(RT_E_ARG, "lambda2 is not finite");
    if ((rc = check_dev_ptr(pin, 4 * n4_of(p.g), "p"))) return rc;
    if ((rc = check_dev_ptr(f_out, nf_of(p.g), "f_out"))) return rc;
    return launch_tv_div(p, pin, lambda2, f_out, (hipStream_t)stream);
}

extern "C" int shrink(const rt_plan *plan, float *pio, float lambda1, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if (!(lambda1 >= 0.f) || !std::isfinite(lambda1))
        return fail(RT_E_ARG, "lambda1 must be finite and >= 0");
    if ((rc = check_dev_ptr(pio, 4 * n4_of(p.g), "p"))) return rc;
    return launch_shrink(p, pio, lambda1, n4_of(p.g), (hipStream_t)stream);
}

extern "C" int rt_fbp_filter(const rt_plan *plan, const float *g, float *q, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if ((rc = check_dev_ptr(g, ng_of(p.g), "g"))) return rc;
    if ((rc = check_dev_ptr(q, ng_of(p.g), "q"))) return rc;
    return launch_fbp_filter(p, g, q, (hipStream_t)stream);
}

extern "C" int rt_fbp(const rt_plan *plan, const float *g, float *f_out, void *stream)
{
    int rc = prologue(plan);
    if (rc) return rc;
    const Plan &p = plan->impl;
    if ((rc = check_dev_ptr(g, ng_of(p.g), "g"))) return rc;
    if ((rc = check_dev_ptr(f_out, nf_of(p.g), "f_out"))) return rc;
    return fbp_init(p, g, f_out, (hipStream_t)stream);
}

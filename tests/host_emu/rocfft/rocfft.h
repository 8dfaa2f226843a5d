// CPU stand-in for the rocFFT declarations used by the library host code.
#pragma once
#include <cstddef>
typedef enum { rocfft_status_success = 0, rocfft_status_failure = 1 } rocfft_status;
typedef enum { rocfft_placement_inplace = 0, rocfft_placement_notinplace = 1 } rocfft_result_placement;
typedef enum { rocfft_transform_type_complex_forward, rocfft_transform_type_complex_inverse,
               rocfft_transform_type_real_forward, rocfft_transform_type_real_inverse } rocfft_transform_type;
typedef enum { rocfft_precision_single, rocfft_precision_double } rocfft_precision;
struct MockPlan; struct MockInfo; struct MockDesc;
typedef MockPlan* rocfft_plan;
typedef MockInfo* rocfft_execution_info;
typedef MockDesc* rocfft_plan_description;
rocfft_status rocfft_setup();
rocfft_status rocfft_plan_create(rocfft_plan*, rocfft_result_placement, rocfft_transform_type, rocfft_precision,
                                 size_t, const size_t*, size_t, const rocfft_plan_description);
rocfft_status rocfft_plan_destroy(rocfft_plan);
rocfft_status rocfft_plan_get_work_buffer_size(const rocfft_plan, size_t*);
rocfft_status rocfft_execution_info_create(rocfft_execution_info*);
rocfft_status rocfft_execution_info_destroy(rocfft_execution_info);
rocfft_status rocfft_execution_info_set_stream(rocfft_execution_info, void*);
rocfft_status rocfft_execution_info_set_work_buffer(rocfft_execution_info, void*, size_t);
rocfft_status rocfft_execute(const rocfft_plan, void**, void**, rocfft_execution_info);
